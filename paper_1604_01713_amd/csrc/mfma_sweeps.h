// Matrix-core (MFMA) versions of the three block-Arnoldi sweeps for block
// sizes P = 8 and 16 with real FP64, FP32 or BF16 basis storage, the update
// sweeps also for P = 4 and the dot sweep for P = 1, 2, 4 (templates;
// the instantiations live in their own translation units).  BF16 blocks are
// widened to FP32 as they are loaded; all arithmetic is FP32 or FP64.
//
// Every sweep streams n rows of a few tall-skinny n x P blocks; all dense
// contractions run on v_mfma_*_16x16x4 tiles:
//   * block dot products S = Q^T W   : S^T = W^T Q, contraction over rows
//     (K = 4 rows per instruction), accumulated over the row range of a
//     workgroup;
//   * block-CGS update  W' = W - Q S : (W')^T = W^T + (-S)^T Q^T, contraction
//     over the columns of Q (K = 4 columns per instruction);
//   * Gram matrix W''^T W'' in FP64 (also for FP32 storage).
// Operand layouts of a 16x16x4 instruction (lane l):
//   A[i][k] = lane (i = l % 16, k = l / 16), B[k][j] = lane (k = l / 16, j = l % 16)
//   D[i][j]: FP64 lane l element v holds i = l/16 + 4v, j = l % 16;
//            FP32 lane l element v holds i = 4(l/16) + v, j = l % 16.
// The kernels are templated on the exact number NC of 16-column chunks of Q,
// so that every load and MFMA of a tile is straight-line code.  Loads are
// never conditional and their values never go through a select (the compiler
// would turn such a select into a branch around the load and wait for it
// there): addresses are clamped into the buffers, operand lanes past P or
// past the last column only feed outputs that are never written, and rows
// past n are zeroed after the loads (on the update result, or on the W
// operand of the last, partial tile).
#pragma once

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "bgcr_internal.h"

namespace bgcr {
namespace mx {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

template <class T> struct MX;
template <> struct MX<double> {
    using acc = d4v;
    __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int drow(int l, int v) { return (l >> 4) + 4 * v; }
    // elements v < VN of a D tile can hold a row below P (for every lane)
    template <int P> static constexpr int vn() { return P / 4 < 4 ? P / 4 : 4; }
};
template <> struct MX<float> {
    using acc = f4v;
    __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int l, int v) { return 4 * (l >> 4) + v; }
    template <int P> static constexpr int vn() { return 4; }
};

constexpr int MROWS = 64;  // rows per workgroup tile of the update sweeps (4 waves x 16 rows)

// XCD-aware renumbering: consecutive logical workgroups (adjacent row ranges)
// run on the same XCD, which shares one L2.
__device__ inline int logical_wg() {
    const int w = blockIdx.x, G = gridDim.x;
    if (G % 8 != 0) return w;
    return (w % 8) * (G / 8) + (w / 8);
}

__device__ inline void tile_span(int64_t ntiles, int lw, int64_t& t0, int64_t& t1) {
    t0 = (int64_t)lw * ntiles / gridDim.x;
    t1 = (int64_t)(lw + 1) * ntiles / gridDim.x;
}

// Cross-wave reduction of the dot accumulators and write of the workgroup
// partial: accumulator [g][ch] holds S^T[w][c] for W column w = 16 g +
// drow(l, v) and Q column c = 16 ch + l % 16.  Output part[lw][(w / P) q P +
// c P + w % P] (one q x P slice per W block), nout = nw q P.
template <class T, int P, int NG, int NC>
__device__ inline void write_dot_partials(const typename MX<T>::acc (&acc)[NG][NC], int q, int nw, double* red,
                                          double* part, int lw, int64_t stride = -1) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t nout = stride < 0 ? (int64_t)nw * q * P : stride;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(wave * 4 + v) * 64 + lane] = (double)acc[g][ch][v];
            __syncthreads();
            // thread t -> (v, lane) = (t / 64, t % 64): sum the 4 waves in order
            const int v = t >> 6, l = t & 63;
            const double s = red[(0 * 4 + v) * 64 + l] + red[(1 * 4 + v) * 64 + l] + red[(2 * 4 + v) * 64 + l] +
                             red[(3 * 4 + v) * 64 + l];
            const int w = 16 * g + MX<T>::drow(l, v);
            const int c = ch * 16 + (l & 15);
            if (w < nw * P && c < q)
                part[(int64_t)lw * nout + (int64_t)(w / P) * q * P + (int64_t)c * P + w % P] = s;
        }
    }
}

// Gram accumulator (FP64 MFMA, D[i][j] = G[i][j]) -> part[lw][off + i P + j]
template <int P>
__device__ inline void write_gram_partials(d4v g, double* red, double* part, int lw, int nout, int off = 0) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) red[(wave * 4 + v) * 64 + lane] = g[v];
    __syncthreads();
    const int v = t >> 6, l = t & 63;
    const double s = red[(0 * 4 + v) * 64 + l] + red[(1 * 4 + v) * 64 + l] + red[(2 * 4 + v) * 64 + l] +
                     red[(3 * 4 + v) * 64 + l];
    const int i = MX<double>::drow(l, v), j = l & 15;
    if (i < P && j < P) part[(int64_t)lw * nout + off + i * P + j] = s;
}

// Per-lane source of the row-major ("RC") operand: lane l reads column
// c = 16 ch + l % 16 of [Q_0 .. Q_{nq-1}], i.e. column c % P of block c / P
// (a 16-column chunk spans 16 / P blocks).  Columns past the last block read
// block 0 (their dot products are never written).  Block pointers are read
// with compile-time indices only (wave-uniform scalar loads) and the lane's
// one is picked by selects, once per kernel.
template <class T, int P, int NC>
__device__ inline void rc_pointers(const T* (&qp)[NC], const BlockPtrs& Q, int nq, int lane) {
    static_assert(P == 1 || P == 2 || P == 4 || P == 8 || P == 16, "block width");
    constexpr int BPC = 16 / P;  // blocks per 16-column chunk
    static_assert(NC * BPC <= MAXB, "chunks beyond the block list");
    const int cl = lane & 15;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
        const T* sel = (const T*)Q.p[0];
#pragma unroll
        for (int u = 0; u < BPC; ++u) {
            const int b = BPC * ch + u;
            const T* pb = (const T*)(b < nq ? Q.p[b] : Q.p[0]);
            sel = (cl / P == u) ? pb : sel;
        }
        qp[ch] = sel + (cl % P);
    }
}

__device__ inline int64_t clamp_row(int64_t row, int64_t n) { return row < n ? row : n - 1; }

// RC operands of KS groups of 4 rows from rbase: [ks][ch] holds
// Q[rbase + 4 ks + l / 16][16 ch + l % 16] (rows clamped to n - 1), stored as
// TS, in the arithmetic type T
template <class T, class TS, int P, int NC, int KS>
__device__ inline void load_rc(T (&qv)[KS][NC], const TS* const (&qp)[NC], int64_t rbase, int64_t n, int lane) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int64_t off = clamp_row(rbase + 4 * ks + (lane >> 4), n) * P;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) qv[ks][ch] = as<T>(qp[ch][off]);
    }
}

// W^T tile in the D layout for rows rbase .. rbase + 15 (rows clamped; D rows
// past P repeat row b % P)
template <class T, int P>
__device__ inline typename MX<T>::acc load_wt(const T* __restrict__ W, int64_t rbase, int64_t n, int lane) {
    typename MX<T>::acc d = typename MX<T>::acc{0, 0, 0, 0};
    const int64_t off = clamp_row(rbase + (lane & 15), n) * P;
#pragma unroll
    for (int v = 0; v < MX<T>::template vn<P>(); ++v) d[v] = W[off + (MX<T>::drow(lane, v) & (P - 1))];
    return d;
}

// zero a D-layout tile in the rows (j = l % 16) at or past n
template <class T>
__device__ inline void zero_tail(typename MX<T>::acc& d, int64_t rbase, int64_t n, int lane) {
    const bool rok = rbase + (lane & 15) < n;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = rok ? d[v] : (T)0;
}

// D-layout tile -> row-major 16 x P in LDS
template <class T, int P>
__device__ inline void d_to_lds(const typename MX<T>::acc& d, T* tr, int lane) {
#pragma unroll
    for (int v = 0; v < MX<T>::template vn<P>(); ++v) {
        const int b = MX<T>::drow(lane, v);
        if (b < P) tr[(lane & 15) * P + b] = d[v];
    }
}

// Row-major 16 x P tile in LDS -> rows rbase .. rbase + 15 of Y (type TO),
// 16 bytes of T per lane and row piece, so that a wave store instruction
// writes whole rows
template <class T, class TO, int P>
__device__ inline void store_tile(const T* tr, TO* __restrict__ Y, int64_t rbase, int64_t n, int lane) {
    constexpr int VT = 16 / (int)sizeof(T), LPRW = P / VT, RPI = 64 / LPRW;  // lanes per row, rows per instruction
    static_assert(P % VT == 0 && 64 % LPRW == 0, "16-byte pieces of a row");
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += RPI) {
        const int r = r0 + lane / LPRW, c = (lane % LPRW) * VT;
        const int64_t row = rbase + r;
        if (r < 16 && row < n) {
            T v[VT];
            __builtin_memcpy(v, tr + r * P + c, 16);
            if constexpr (std::is_same<TO, T>::value) {
                __builtin_memcpy(Y + row * P + c, v, 16);
            } else {
                TO o[VT];
#pragma unroll
                for (int u = 0; u < VT; ++u) o[u] = to_store<TO>(v[u]);
                __builtin_memcpy(Y + row * P + c, o, sizeof(o));
            }
        }
    }
}

// Wave-private LDS tile of 16 rows x QLD columns (QLD a multiple of 32),
// XOR-swizzled on column bits 2..4 so that both the row-major (4 rows x 16
// columns) and the column-major (16 rows x 4 columns) accesses of a wave
// spread evenly over the banks.
template <int QLD>
__device__ inline int qsw(int r, int c) {
    const int s = ((r & 1) << 2) | ((r >> 1) & 3);
    return r * QLD + (c ^ (s << 2));
}

// ---------------------------------------------------------------------------
// dot sweep: partial S^T = [W_0 .. W_{nw-1}]^T [Q_0 .. Q_{nq-1}] (no update),
// NG groups of 16 W columns (two W blocks per group for P = 8).  Both MFMA
// operands are loaded from global memory directly in their register layout
// (A = W[row][w], B = Q[row][c], 4 rows per instruction), so the sweep needs
// no LDS besides the final cross-wave reduction; the next wave tile is loaded
// while the current one is multiplied.
// ---------------------------------------------------------------------------
template <class T, class TW, class TQ, int P, int NC, int KS, int NG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && NC * NG > 18 ? 1 : 2))) void
k_dot_mfma(int64_t n, BlockPtrs W, int nw, BlockPtrs Q, int nq, double* __restrict__ part, const Ctl* ctl, int rev) {
    using M = MX<T>;
    constexpr int WROWS = 4 * KS, TROWS = 4 * WROWS;
    if (ctl && ctl->active == 0) return;
    const int q = nq * P;
    extern __shared__ __align__(16) unsigned char smem[];
    double* red = (double*)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const TQ* qp[NC];
    rc_pointers<TQ, P, NC>(qp, Q, nq, lane);
    const TW* wp[NG];
    rc_pointers<TW, P, NG>(wp, W, nw, lane);
    typename M::acc acc[NG][NC];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) acc[g][ch] = typename M::acc{0, 0, 0, 0};
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + TROWS - 1) / TROWS, lw, t0, t1);
    const int64_t cnt = t1 - t0, dstep = rev ? -TROWS : TROWS;
    T qn[KS][NC], wn[KS][NG];
    if (cnt > 0) {
        const int64_t r0 = (rev ? t1 - 1 : t0) * TROWS + wave * WROWS;
        load_rc<T, TQ, P, NC, KS>(qn, qp, r0, n, lane);
        load_rc<T, TW, P, NG, KS>(wn, wp, r0, n, lane);
    }
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t tile = rev ? t1 - 1 - k : t0 + k;
        const int64_t rbase = tile * TROWS + wave * WROWS;
        T qc[KS][NC], wc[KS][NG];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int g = 0; g < NG; ++g) wc[ks][g] = wn[ks][g];
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) qc[ks][ch] = qn[ks][ch];
        }
        if (rbase + WROWS > n) {  // last, partial tile: rows past n contribute nothing
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int g = 0; g < NG; ++g) wc[ks][g] = rbase + 4 * ks + (lane >> 4) < n ? wc[ks][g] : (T)0;
        }
        if (k + 1 < cnt) {
            load_rc<T, TQ, P, NC, KS>(qn, qp, rbase + dstep, n, lane);
            load_rc<T, TW, P, NG, KS>(wn, wp, rbase + dstep, n, lane);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) acc[g][ch] = M::mma(wc[ks][g], qc[ks][ch], acc[g][ch]);
    }
    write_dot_partials<T, P, NG, NC>(acc, q, nw, red, part, lw);
}

// ---------------------------------------------------------------------------
// update-and-dot sweep: W' = W - Q S (not stored); partial S' = Q^T W' and,
// with GRAM, partial W'^T W' (FP64) after it (partial layout [q P dots][P P]).
// Q is loaded row-major, staged in a wave-private LDS tile and read back
// column-major for the update and row-major for the dot; the next tile's
// loads are in flight while the current one is computed.  No workgroup
// barrier inside the loop (each wave only reads what it wrote).
// ---------------------------------------------------------------------------
template <class T, class TQ, int P, int NC, bool GRAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 8 ? NC <= 7 : NC <= 10) ? 2 : 1))) void k_proj_dot_mfma(
    int64_t n, const T* __restrict__ Win, BlockPtrs Q, int nq, const double* __restrict__ S, double* __restrict__ part,
    const Ctl* ctl, int rev) {
    using M = MX<T>;
    constexpr int NQ = NC * 16 / P, KK = P / 4, QLD = 32 * ((NC + 1) / 2);
    if (ctl && ctl->active == 0) return;
    const int q = nq * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T* Ss = (T*)smem;                        // [NQ*P][P]: -S, zero past q
    T* Qt = Ss + NQ * P * P;                 // [4 waves][16][QLD]
    T* Wt = Qt + 4 * 16 * QLD;               // [4 waves][16][P]
    double* red = (double*)smem;             // reused at the end: 1024 doubles
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int bl = lane & 15, rq = lane >> 4, bc = bl & (P - 1);
    for (int e = t; e < NQ * P * P; e += 256) Ss[e] = (e < q * P) ? (T)(-S[e]) : (T)0;
    const TQ* qp[NC];
    rc_pointers<TQ, P, NC>(qp, Q, nq, lane);
    typename M::acc acc[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[ch] = typename M::acc{0, 0, 0, 0};
    d4v gacc = {0, 0, 0, 0};
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    T* myQ = Qt + wave * 16 * QLD;
    T* myW = Wt + wave * 16 * P;
    T qn[4][NC];
    typename M::acc wn = typename M::acc{0, 0, 0, 0};
    const int64_t cnt = t1 - t0, dstep = rev ? -MROWS : MROWS;
    if (cnt > 0) {
        const int64_t r0 = (rev ? t1 - 1 : t0) * MROWS + wave * 16;
        load_rc<T, TQ, P, NC, 4>(qn, qp, r0, n, lane);
        wn = load_wt<T, P>(Win, r0, n, lane);
    }
    __syncthreads();
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t tile = rev ? t1 - 1 - k : t0 + k;
        const int64_t rbase = tile * MROWS + wave * 16;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) myQ[qsw<QLD>(4 * ks + rq, 16 * ch + bl)] = qn[ks][ch];
        typename M::acc d = wn;
        if (k + 1 < cnt) {
            load_rc<T, TQ, P, NC, 4>(qn, qp, rbase + dstep, n, lane);
            wn = load_wt<T, P>(Win, rbase + dstep, n, lane);
        }
        // D = W^T + (-S)^T Q^T over the columns of Q, 4 per instruction
        // (A rows past P repeat row b % P; those D rows are never stored).
        // FP64 blocks of 8 columns take two 4x4x4 MFMAs (four 4 x 4 blocks
        // each, one per group of 4 rows) per step instead, one for W columns
        // 0..3 and one for 4..7: the same B operand and D elements 0 and 1 of
        // the 16 x 16 layout, without its repeated half.
        constexpr bool DUAL4 = std::is_same<T, double>::value && P == 8;
        if constexpr (DUAL4) {
            double d0 = d[0], d1 = d[1];
#pragma unroll
            for (int blk = 0; blk < NQ; ++blk) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = blk * P + 4 * kk + rq;
                    const double qv = myQ[qsw<QLD>(bl, c)];
                    d0 = __builtin_amdgcn_mfma_f64_4x4x4f64(Ss[c * P + (lane & 3)], qv, d0, 0, 0, 0);
                    d1 = __builtin_amdgcn_mfma_f64_4x4x4f64(Ss[c * P + 4 + (lane & 3)], qv, d1, 0, 0, 0);
                }
            }
            d[0] = d0;
            d[1] = d1;
        } else {
#pragma unroll
            for (int blk = 0; blk < NQ; ++blk) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = blk * P + 4 * kk + rq;
                    d = M::mma(Ss[c * P + bc], myQ[qsw<QLD>(bl, c)], d);
                }
            }
        }
        zero_tail<T>(d, rbase, n, lane);
        d_to_lds<T, P>(d, myW, lane);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rl = 4 * ks + rq;
            const T wv = myW[rl * P + bc];
            if constexpr (DUAL4) {
                // A operand W'[rl][4 h + l % 4] for W column group h
                const double w0 = myW[rl * P + (lane & 3)], w1 = myW[rl * P + 4 + (lane & 3)];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) {
                    const double qv = myQ[qsw<QLD>(rl, 16 * ch + bl)];
                    acc[ch][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(w0, qv, acc[ch][0], 0, 0, 0);
                    acc[ch][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(w1, qv, acc[ch][1], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) acc[ch] = M::mma(wv, myQ[qsw<QLD>(rl, 16 * ch + bl)], acc[ch]);
            }
            if constexpr (GRAM) gacc = MX<double>::mma((double)wv, (double)wv, gacc);
        }
    }
    typename M::acc acc1[1][NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc1[0][ch] = acc[ch];
    const int64_t stride = (int64_t)q * P + (GRAM ? P * P : 0);
    write_dot_partials<T, P, 1, NC>(acc1, q, 1, red, part, lw, stride);
    if constexpr (GRAM) write_gram_partials<P>(gacc, red, part, lw, (int)stride, q * P);
}

// ---------------------------------------------------------------------------
// update-and-Gram sweep: W'' = W - Q S, stored (optional); partial Gram
// W''^T W'' in FP64.  NC = 0: no update (Gram of W only).  With NORM the
// sweep stores V = W'' R^{-1} instead (R^{-1} given, P x P FP64) and computes
// no Gram.  The update operands are loaded column-major straight into
// registers, double-buffered.
// ---------------------------------------------------------------------------
template <class T, class TQ, class TO, int P, int NC, bool NORM>
__global__ __launch_bounds__(256) void k_proj_gram_mfma(int64_t n, const T* Win, BlockPtrs Q, int nq,
                                                        const double* __restrict__ S, TO* Wout,
                                                        double* __restrict__ part, const double* __restrict__ Rinv,
                                                        const Ctl* ctl, int step, int rev) {
    using M = MX<T>;
    constexpr int NQ = NC * 16 / P, KK = P / 4, NQV = NQ * KK, NQA = NQ > 0 ? NQ : 1;
    // runs while the cycle is active, and also for the step at which it just
    // stopped without breakdown (its block V_{step+1} is still needed)
    if (ctl && ctl->active == 0 && !(ctl->meff == step && ctl->status == 0)) return;
    const int q = nq * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T* Ss = (T*)smem;                  // [NQA*P][P]: -S, zero past q
    T* tr = Ss + NQA * P * P;          // [4 waves][16][P]
    double* red = (double*)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int bl = lane & 15, rq = lane >> 4, bc = bl & (P - 1);
    for (int e = t; e < NQA * P * P; e += 256) Ss[e] = (e < q * P) ? (T)(-S[e]) : (T)0;
    const TQ* qb[NQA];
#pragma unroll
    for (int blk = 0; blk < NQA; ++blk) qb[blk] = (const TQ*)(blk < nq ? Q.p[blk] : Q.p[0]);
    d4v gacc = {0, 0, 0, 0};
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    T* mytr = tr + wave * 16 * P;
    // NORM: A operands (R^{-1})^T[b'][b] for b = 4 kk + l/16, b' = l % 16
    // (FP64 blocks of 8 columns: the 4x4x4 operands for b' = l % 4 and 4 + l % 4)
    constexpr bool DUAL4 = std::is_same<T, double>::value && P == 8;
    T ra[KK], rb[KK];
    if constexpr (NORM) {
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            ra[kk] = (T)Rinv[(4 * kk + rq) * P + (DUAL4 ? (lane & 3) : bc)];
            rb[kk] = DUAL4 ? (T)Rinv[(4 * kk + rq) * P + 4 + (lane & 3)] : ra[kk];
        }
    }
    // column-major operands: [blk*KK + kk] holds Q_blk[rbase + l % 16][4 kk + l / 16]
    auto load_cr = [&](T(&qv)[NQA * KK], int64_t rbase) {
        const int64_t off = clamp_row(rbase + bl, n) * P + rq;
#pragma unroll
        for (int blk = 0; blk < NQ; ++blk)
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) qv[blk * KK + kk] = as<T>(qb[blk][off + 4 * kk]);
    };
    T qn[NQA * KK];
    typename M::acc wn = typename M::acc{0, 0, 0, 0};
    const int64_t cnt = t1 - t0, dstep = rev ? -MROWS : MROWS;
    if (cnt > 0) {
        const int64_t r0 = (rev ? t1 - 1 : t0) * MROWS + wave * 16;
        if constexpr (NQV > 0) load_cr(qn, r0);
        wn = load_wt<T, P>(Win, r0, n, lane);
    }
    __syncthreads();
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t tile = rev ? t1 - 1 - k : t0 + k;
        const int64_t rbase = tile * MROWS + wave * 16;
        typename M::acc d = wn;
        if constexpr (NQV > 0) {
            T qc[NQA * KK];
#pragma unroll
            for (int e = 0; e < NQV; ++e) qc[e] = qn[e];
            if (k + 1 < cnt) load_cr(qn, rbase + dstep);
            if constexpr (DUAL4) {
                // two four-block 4x4x4 MFMAs per step (W columns 0..3, 4..7):
                // D elements 0 and 1 of the 16x16x4 layout without its repeats
                double d0 = d[0], d1 = d[1];
#pragma unroll
                for (int blk = 0; blk < NQ; ++blk) {
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk) {
                        const T* sr = Ss + (blk * P + 4 * kk + rq) * P;
                        d0 = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[lane & 3], qc[blk * KK + kk], d0, 0, 0, 0);
                        d1 = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[4 + (lane & 3)], qc[blk * KK + kk], d1, 0, 0, 0);
                    }
                }
                d[0] = d0;
                d[1] = d1;
            } else {
#pragma unroll
                for (int blk = 0; blk < NQ; ++blk) {
#pragma unroll
                    for (int kk = 0; kk < KK; ++kk)
                        d = M::mma(Ss[(blk * P + 4 * kk + rq) * P + bc], qc[blk * KK + kk], d);
                }
            }
        }
        if (k + 1 < cnt) wn = load_wt<T, P>(Win, rbase + dstep, n, lane);
        const int64_t row = rbase + bl;
        zero_tail<T>(d, rbase, n, lane);
        if constexpr (NORM) {
            // V^T = (R^{-1})^T W''^T: B operand W''^T[4 kk + l/16][row l % 16] from the tile in LDS
            d_to_lds<T, P>(d, mytr, lane);
            typename M::acc dv = typename M::acc{0, 0, 0, 0};
            if constexpr (DUAL4) {
                double v0 = 0.0, v1 = 0.0;
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const double wv = mytr[bl * P + 4 * kk + rq];
                    v0 = __builtin_amdgcn_mfma_f64_4x4x4f64(ra[kk], wv, v0, 0, 0, 0);
                    v1 = __builtin_amdgcn_mfma_f64_4x4x4f64(rb[kk], wv, v1, 0, 0, 0);
                }
                dv[0] = v0;
                dv[1] = v1;
            } else {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) dv = M::mma(ra[kk], mytr[bl * P + 4 * kk + rq], dv);
            }
            if (row < n) {
#pragma unroll
                for (int v = 0; v < M::template vn<P>(); ++v) {
                    const int b = M::drow(lane, v);
                    if (b < P) Wout[row * P + b] = to_store<TO>(dv[v]);
                }
            }
        } else {
            if (Wout && row < n) {
#pragma unroll
                for (int v = 0; v < M::template vn<P>(); ++v) {
                    const int b = M::drow(lane, v);
                    if (b < P) Wout[row * P + b] = to_store<TO>(d[v]);
                }
            }
            d_to_lds<T, P>(d, mytr, lane);
            // Gram rows and columns past P repeat column b % P and are never written
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const double wv = (double)mytr[(4 * ks + rq) * P + bc];
                gacc = MX<double>::mma(wv, wv, gacc);
            }
        }
    }
    if constexpr (!NORM) write_gram_partials<P>(gacc, red, part, lw, P * P);
}

// ---------------------------------------------------------------------------
// Wide tile loads: a wave's 16-row tile of [Q_0 .. Q_{NQ-1}] is read with
// 16-byte loads (V = 16 / sizeof(TS) consecutive columns of one row of one
// block per lane), so that every wave load instruction moves 1 KB whatever
// the storage type; the tile is written to the wave-private LDS tile in the
// arithmetic type T and the MFMA operands are read back from there.
// ---------------------------------------------------------------------------

template <class TS, int P, int NQ>
struct Wide {
    static constexpr int V = 16 / (int)sizeof(TS);  // columns per lane and load
    static constexpr int LPR = P / V;               // lanes per row of a block
    static constexpr int LPB = 16 * LPR;            // lanes per 16-row block tile
    static constexpr int NI = (NQ * LPB + 63) / 64; // loads per lane per tile
    static constexpr int NIA = NI > 0 ? NI : 1;
    static_assert(P % V == 0, "a lane's 16 bytes lie in one row of a block");
    static_assert(LPB >= 64 ? LPB % 64 == 0 : 64 % LPB == 0, "block tiles align with waves");
};

// block, row and first column of load i of this lane
template <class TS, int P, int NQ>
__device__ inline void wide_slot(int i, int lane, int& blk, int& r, int& c0) {
    using Wd = Wide<TS, P, NQ>;
    const int slot = i * 64 + lane;
    blk = slot / Wd::LPB;
    const int rem = slot % Wd::LPB;
    r = rem / Wd::LPR;
    c0 = blk * P + (rem % Wd::LPR) * Wd::V;
}

template <class TS, int P, int NQ>
__device__ inline void wide_load(u4v* buf, const TS* const* qb, int64_t rbase, int64_t n, int lane) {
    using Wd = Wide<TS, P, NQ>;
#pragma unroll
    for (int i = 0; i < Wd::NI; ++i) {
        int blk, r, c0;
        wide_slot<TS, P, NQ>(i, lane, blk, r, c0);
        // the block pointer is picked among compile-time candidates (a select
        // of addresses, not of loaded values); slots past the last block
        // reload the last block and are not written to LDS
        const TS* p;
        if constexpr (Wd::LPB >= 64) {
            p = qb[(i * 64) / Wd::LPB];
        } else {
            constexpr int G = 64 / Wd::LPB;
            const int g = lane / Wd::LPB;
            p = qb[(i * G) < NQ ? i * G : NQ - 1];
#pragma unroll
            for (int gg = 1; gg < G; ++gg) {
                const TS* pg = qb[(i * G + gg) < NQ ? i * G + gg : NQ - 1];
                p = g == gg ? pg : p;
            }
        }
        const int64_t off = clamp_row(rbase + r, n) * P + (c0 - blk * P);
        buf[i] = *(const u4v*)(p + off);
    }
}

// write the loaded tile to the wave-private LDS tile [16][QLD] in type T
// (T at least as wide as TS), 16 bytes per LDS write; 16-byte groups of
// columns stay contiguous under the swizzle (it changes bits 2..4 only)
template <class T, class TS, int P, int NQ, int QLD>
__device__ inline void wide_to_lds(T* myQ, const u4v* buf, int lane) {
    using Wd = Wide<TS, P, NQ>;
    constexpr int V = Wd::V, VT = 16 / (int)sizeof(T);
    static_assert(sizeof(TS) <= sizeof(T), "tiles are widened, never narrowed");
#pragma unroll
    for (int i = 0; i < Wd::NI; ++i) {
        int blk, r, c0;
        wide_slot<TS, P, NQ>(i, lane, blk, r, c0);
        if ((NQ * Wd::LPB) % 64 != 0 && blk >= NQ) continue;
        TS e[V];
        __builtin_memcpy(e, &buf[i], 16);
#pragma unroll
        for (int h = 0; h < V; h += VT) {
            T o[VT];
#pragma unroll
            for (int u = 0; u < VT; ++u) o[u] = as<T>(e[h + u]);
            u4v w;
            __builtin_memcpy(&w, o, 16);
            *(u4v*)(myQ + qsw<QLD>(r, c0 + h)) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// One sweep of a block step over n rows, on 16-row wave tiles:
//   D = W (UPD: D = W - Q S);
//   NORM: store V = D R^{-1} (as TO);
//   otherwise store D (Wout non-null), partial dots Q^T D (DOT) and partial
//   Gram D^T D in FP64 (GRAM) (partial layout [q P dots][P P]).
// Q is read with wide loads into the wave-private LDS tile (the next tile's
// loads in flight while the current one is computed) and read back
// column-major for the update and row-major for the dots; no workgroup
// barrier inside the loop (each wave only reads what it wrote).  With a
// control block the sweep runs while the cycle is active and also for block
// step `step` if the cycle just stopped there without breakdown.
// ---------------------------------------------------------------------------
template <class T, int P, int NC, class TQ, bool UPD, bool DOT>
constexpr int sweep_waves() {
    // two waves per SIMD up to the chunk counts at which the FP32 variants
    // still compile without spills at 256 registers; one wave above
    return NC <= (UPD && DOT ? (sizeof(T) == 8 ? 6 : (sizeof(TQ) == 2 ? 11 : 9)) : 14) ? 2 : 1;
}

template <class T, class TQ, class TO, int P, int NC, bool UPD, bool DOT, bool GRAM, bool NORM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_waves<T, P, NC, TQ, UPD, DOT>()))) void
k_sweep_mfma(int64_t n, const T* Win, BlockPtrs Q, int nq, const double* __restrict__ S,
             TO* Wout, double* __restrict__ part, const double* __restrict__ Rinv, const Ctl* ctl,
             int step) {
    using M = MX<T>;
    constexpr int NQ = NC * 16 / P, NQA = NQ > 0 ? NQ : 1, KK = P / 4, QLD = 32 * ((NC + 1) / 2);
    constexpr bool TILE = NQ > 0 && (UPD || DOT);
    using Wd = Wide<TQ, P, NQ>;
    static_assert(!(NORM && (DOT || GRAM)), "the normalising sweep stores V only");
    if (ctl && ctl->active == 0 && !(ctl->meff == step && ctl->status == 0)) return;
    const int q = nq * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T* Ss = (T*)smem;                            // [NQ*P][P]: -S, zero past q (UPD)
    T* Qt = Ss + (UPD ? NQA * P * P : 0);        // [4 waves][16][QLD] (TILE)
    T* Wt = Qt + (TILE ? 4 * 16 * QLD : 0);      // [4 waves][16][P]
    double* red = (double*)smem;                 // reused at the end: 1024 doubles
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int bl = lane & 15, rq = lane >> 4, bc = bl & (P - 1);
    if constexpr (UPD) {
        for (int e = t; e < NQA * P * P; e += 256) Ss[e] = (e < q * P) ? (T)(-S[e]) : (T)0;
    }
    const TQ* qb[NQA];
#pragma unroll
    for (int blk = 0; blk < NQA; ++blk) qb[blk] = (const TQ*)(blk < nq ? Q.p[blk] : Q.p[0]);
    constexpr int NACC = DOT && NC > 0 ? NC : 1;
    typename M::acc acc[NACC];
#pragma unroll
    for (int ch = 0; ch < NACC; ++ch) acc[ch] = typename M::acc{0, 0, 0, 0};
    d4v gacc = {0, 0, 0, 0};
    T ra[KK];
    if constexpr (NORM) {
        // A operands (R^{-1})^T[b'][b] for b = 4 kk + l/16, b' = l % 16
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) ra[kk] = (T)Rinv[(4 * kk + rq) * P + bc];
    }
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    T* myQ = Qt + wave * 16 * QLD;
    T* myW = Wt + wave * 16 * P;
    u4v qn[Wd::NIA];
    typename M::acc wn = typename M::acc{0, 0, 0, 0};
    if (t0 < t1) {
        if constexpr (TILE) wide_load<TQ, P, NQ>(qn, qb, t0 * MROWS + wave * 16, n, lane);
        wn = load_wt<T, P>(Win, t0 * MROWS + wave * 16, n, lane);
    }
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t rbase = tile * MROWS + wave * 16;
        if constexpr (TILE) wide_to_lds<T, TQ, P, NQ, QLD>(myQ, qn, lane);
        typename M::acc d = wn;
        if (tile + 1 < t1) {
            if constexpr (TILE) wide_load<TQ, P, NQ>(qn, qb, rbase + MROWS, n, lane);
            wn = load_wt<T, P>(Win, rbase + MROWS, n, lane);
        }
        if constexpr (UPD && NQ > 0) {
            // D = W^T + (-S)^T Q^T over the columns of Q, 4 per instruction
            // (A rows past P repeat row b % P; those D rows are never stored)
#pragma unroll
            for (int blk = 0; blk < NQ; ++blk) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = blk * P + 4 * kk + rq;
                    d = M::mma(Ss[c * P + bc], myQ[qsw<QLD>(bl, c)], d);
                }
            }
        }
        zero_tail<T>(d, rbase, n, lane);
        const int64_t row = rbase + bl;
        if constexpr (NORM) {
            // V^T = (R^{-1})^T W''^T: B operand W''^T[4 kk + l/16][row l % 16] from LDS
            d_to_lds<T, P>(d, myW, lane);
            typename M::acc dv = typename M::acc{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) dv = M::mma(ra[kk], myW[bl * P + 4 * kk + rq], dv);
            // (the wave's LDS operations run in order: the tile is read above before it is overwritten)
            d_to_lds<T, P>(dv, myW, lane);
            store_tile<T, TO, P>(myW, Wout, rbase, n, lane);
        } else {
            if (Wout && row < n) {
#pragma unroll
                for (int v = 0; v < M::template vn<P>(); ++v) {
                    const int b = M::drow(lane, v);
                    if (b < P) Wout[row * P + b] = to_store<TO>(d[v]);
                }
            }
            if constexpr (DOT || GRAM) {
                d_to_lds<T, P>(d, myW, lane);
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int rl = 4 * ks + rq;
                    const T wv = myW[rl * P + bc];
                    if constexpr (DOT && NQ > 0) {
#pragma unroll
                        for (int ch = 0; ch < NC; ++ch) acc[ch] = M::mma(wv, myQ[qsw<QLD>(rl, 16 * ch + bl)], acc[ch]);
                    }
                    // Gram rows and columns past P repeat column b % P and are never written
                    if constexpr (GRAM) gacc = MX<double>::mma((double)wv, (double)wv, gacc);
                }
            }
        }
    }
    const int64_t stride = (DOT ? (int64_t)q * P : 0) + (GRAM ? P * P : 0);
    if constexpr (DOT && NQ > 0) {
        typename M::acc acc1[1][NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) acc1[0][ch] = acc[ch];
        write_dot_partials<T, P, 1, NC>(acc1, q, 1, red, part, lw, stride);
    }
    if constexpr (GRAM) write_gram_partials<P>(gacc, red, part, lw, (int)stride, DOT ? q * P : 0);
}

// ---------------------------------------------------------------------------
// launchers: hipErrorNotSupported when the shape has no MFMA variant
// ---------------------------------------------------------------------------
template <class F>
inline void allow_lds(F* f) {
    (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// dispatch on the exact chunk count nc (1..16)
#define BGCR_MX_NC_DISPATCH(nc, MACRO) \
    switch (nc) {                      \
        case 1: MACRO(1); break;       \
        case 2: MACRO(2); break;       \
        case 3: MACRO(3); break;       \
        case 4: MACRO(4); break;       \
        case 5: MACRO(5); break;       \
        case 6: MACRO(6); break;       \
        case 7: MACRO(7); break;       \
        case 8: MACRO(8); break;       \
        case 9: MACRO(9); break;       \
        case 10: MACRO(10); break;     \
        case 11: MACRO(11); break;     \
        case 12: MACRO(12); break;     \
        case 13: MACRO(13); break;     \
        case 14: MACRO(14); break;     \
        case 15: MACRO(15); break;     \
        case 16: MACRO(16); break;     \
        default: return hipErrorNotSupported; \
    }

// rows per wave tile of the dot sweep (4 KS) so that the double-buffered
// operands keep two waves per SIMD
template <int NC>
constexpr int dot_ks() {
    return NC <= 8 ? 4 : (NC <= 12 ? 2 : 1);
}

template <class T, class TW, class TQ, int P>
hipError_t launch_dot(hipStream_t st, int64_t n, const BlockPtrs& W, int nw, const BlockPtrs& Q, int nq, double* part,
                      int nwg, const Ctl* ctl, bool rev = false) {
    const int nc = (nq * P + 15) / 16, ng = (nw * P + 15) / 16;
    const size_t lds = (size_t)1024 * sizeof(double);
    // a chunk of narrow blocks spans 16 / P block pointers: at most MAXB in all
    if (nc * (16 / P) > MAXB || ng * (16 / P) > MAXB) return hipErrorNotSupported;
    if (ng == 1) {
#define L(NC)                                                                                                      \
    if constexpr ((NC) * (16 / P) <= MAXB)                                                                         \
        hipLaunchKernelGGL((k_dot_mfma<T, TW, TQ, P, NC, dot_ks<NC>(), 1>), dim3(nwg), dim3(256), lds, st, n, W, nw, Q, nq, \
                           part, ctl, (int)rev)
        BGCR_MX_NC_DISPATCH(nc, L)
#undef L
    } else if (ng == 2 && nc <= 9) {
#define L(NC)                                                                                                      \
    if constexpr ((NC) * (16 / P) <= MAXB)                                                                         \
        hipLaunchKernelGGL((k_dot_mfma<T, TW, TQ, P, NC, dot_ks<2 * NC>(), 2>), dim3(nwg), dim3(256), lds, st, n, W, nw, Q, \
                           nq, part, ctl, (int)rev)
        switch (nc) {
            case 1: L(1); break;
            case 2: L(2); break;
            case 3: L(3); break;
            case 4: L(4); break;
            case 5: L(5); break;
            case 6: L(6); break;
            case 7: L(7); break;
            case 8: L(8); break;
            case 9: L(9); break;
            default: return hipErrorNotSupported;
        }
#undef L
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <class T, class TQ, int P, bool GRAM>
hipError_t launch_proj_dot_t(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                             double* part, int nwg, const Ctl* ctl, bool rev) {
    const int nc = (nq * P + 15) / 16;
#define L(NC)                                                                                                   \
    {                                                                                                           \
        constexpr int NQ = NC * 16 / P, QLD = 32 * ((NC + 1) / 2);                                              \
        const size_t lds = std::max((size_t)(NQ * P * P + 4 * 16 * QLD + 4 * 16 * P) * sizeof(T),                \
                                    (size_t)1024 * sizeof(double));                                             \
        if (lds > (size_t)160 * 1024) return hipErrorNotSupported;                                              \
        static std::once_flag fl;                                                                               \
        std::call_once(fl, [] { allow_lds(k_proj_dot_mfma<T, TQ, P, NC, GRAM>); });                             \
        hipLaunchKernelGGL((k_proj_dot_mfma<T, TQ, P, NC, GRAM>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S, \
                           part, ctl, (int)rev);                                                                \
    }
    BGCR_MX_NC_DISPATCH(nc, L)
#undef L
    return hipGetLastError();
}

template <class T, class TQ, int P>
hipError_t launch_proj_dot(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                           double* part, int nwg, const Ctl* ctl, bool gram, bool rev = false) {
    return gram ? launch_proj_dot_t<T, TQ, P, true>(st, n, Win, Q, nq, S, part, nwg, ctl, rev)
                : launch_proj_dot_t<T, TQ, P, false>(st, n, Win, Q, nq, S, part, nwg, ctl, rev);
}

template <class T, class TQ, class TO, int P, bool NORM>
hipError_t launch_proj_gram_t(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                              TO* Wout, double* part, const double* Rinv, int nwg, const Ctl* ctl, int step, bool rev) {
    const int nc = (nq * P + 15) / 16;
#define L(NC)                                                                                                    \
    {                                                                                                            \
        constexpr int NQA = NC * 16 / P > 0 ? NC * 16 / P : 1;                                                   \
        const size_t lds = std::max((size_t)(NQA * P * P + 4 * 16 * P) * sizeof(T), (size_t)1024 * sizeof(double)); \
        hipLaunchKernelGGL((k_proj_gram_mfma<T, TQ, TO, P, NC, NORM>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S, \
                           Wout, part, Rinv, ctl, step, (int)rev);                                               \
    }
    if (nq == 0) {
        L(0);
        return hipGetLastError();
    }
    BGCR_MX_NC_DISPATCH(nc, L)
#undef L
    return hipGetLastError();
}

template <class T, class TQ, class TO, int P>
hipError_t launch_proj_gram(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                            TO* Wout, double* part, const double* Rinv, int nwg, const Ctl* ctl, int step,
                            bool rev = false) {
    return Rinv ? launch_proj_gram_t<T, TQ, TO, P, true>(st, n, Win, Q, nq, S, Wout, part, Rinv, nwg, ctl, step, rev)
                : launch_proj_gram_t<T, TQ, TO, P, false>(st, n, Win, Q, nq, S, Wout, part, Rinv, nwg, ctl, step, rev);
}


// ---------------------------------------------------------------------------
// block combination, FP64 inputs: as k_combine_mfma below (FP64 arithmetic)
// with the A operands loaded straight into registers instead of through an
// LDS tile, which keeps the LDS to the coefficients (two workgroups per CU at
// 64 output columns).
// A = X[row][k] (column-major operand loads straight into registers, G input
// blocks per pipeline step, the next step's loads in flight while the current
// one is multiplied; the step sequence runs across row tiles), B = C[k][j]
// from LDS, padded to NCO chunks of 16 output columns.
// ---------------------------------------------------------------------------
// CX: complex blocks of P / 2 columns seen as real blocks of P interleaved
// (re, im) columns, and complex coefficients ((K / 2) x (N / 2), row-major):
// the real coefficient C_r[k][j] is the real part of the complex entry
// (k / 2, j / 2) where k and j have the same parity, else its imaginary part,
// negated for (k odd, j even); the LDS holds the complex matrix.
template <class TI, class TO, int P, int NCO, bool CX = false>
__global__ __launch_bounds__(256) void k_combine_scalar(int64_t n, BlockPtrs in, int nin, BlockPtrs out, int nout,
                                                      const double* __restrict__ coef, int accumulate) {
    using M = MX<double>;
    constexpr int KK = P / 4, G = 64 / P, NV = G * KK, NPAD = 16 * NCO;
    const int N = nout * P, K = nin * P;
    extern __shared__ __align__(16) unsigned char smem[];
    double* Cs = (double*)smem;  // [K][NPAD], or with CX [K/2][NPAD/2] complex
    if constexpr (CX) {
        const int Nc = N / 2, NPc = NPAD / 2;
        for (int e = threadIdx.x; e < (K / 2) * NPc; e += 256) {
            const int k = e / NPc, j = e % NPc;
            const bool ok = j < Nc;
            Cs[2 * e] = ok ? coef[2 * ((int64_t)k * Nc + j)] : 0.0;
            Cs[2 * e + 1] = ok ? coef[2 * ((int64_t)k * Nc + j) + 1] : 0.0;
        }
    } else {
        for (int e = threadIdx.x; e < K * NPAD; e += 256) {
            const int k = e / NPAD, j = e % NPAD;
            Cs[e] = j < N ? coef[(int64_t)k * N + j] : 0.0;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, bl = lane & 15, rq = lane >> 4;
    const int ol = (rq ^ bl) & 1;
    const double sg = (CX && (rq & 1) && !(bl & 1)) ? -1.0 : 1.0;
    const int nch = (nin + G - 1) / G;
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    const int64_t nsteps = (t1 - t0) * nch;
    auto load = [&](double(&v)[NV], int64_t s) {
        const int64_t tile = t0 + s / nch;
        const int c = (int)(s % nch);
        const int64_t off = clamp_row(tile * MROWS + wave * 16 + bl, n) * P + rq;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int blk = c * G + g;
            const TI* p = (const TI*)in.p[blk < nin ? blk : 0];
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) v[g * KK + kk] = as<double>(p[off + 4 * kk]);
        }
    };
    typename M::acc acc[NCO];
#pragma unroll
    for (int oc = 0; oc < NCO; ++oc) acc[oc] = typename M::acc{0, 0, 0, 0};
    double an[NV];
    if (nsteps > 0) load(an, 0);
    for (int64_t s = 0; s < nsteps; ++s) {
        double ac[NV];
#pragma unroll
        for (int e = 0; e < NV; ++e) ac[e] = an[e];
        if (s + 1 < nsteps) load(an, s + 1);
        const int c = (int)(s % nch);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int blk = c * G + g;
            if (blk < nin) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    if constexpr (CX) {
                        const double* cr = Cs + ((blk * P + 4 * kk + rq) >> 1) * NPAD + 2 * (bl >> 1) + ol;
#pragma unroll
                        for (int oc = 0; oc < NCO; ++oc) acc[oc] = M::mma(ac[g * KK + kk], sg * cr[16 * oc], acc[oc]);
                    } else {
                        const double* cr = Cs + (blk * P + 4 * kk + rq) * NPAD + bl;
#pragma unroll
                        for (int oc = 0; oc < NCO; ++oc) acc[oc] = M::mma(ac[g * KK + kk], cr[16 * oc], acc[oc]);
                    }
                }
            }
        }
        if (c == nch - 1) {
            // D[row][col]: lane l element v holds row rbase + l/16 + 4v, column 16 oc + l%16
            const int64_t rbase = (t0 + s / nch) * MROWS + wave * 16;
#pragma unroll
            for (int oc = 0; oc < NCO; ++oc) {
                const int col = 16 * oc + bl;
                const int ob = col / P, b = col % P;
                // output block of this lane's column: one of the 16 / P blocks of the
                // chunk (a 32-column block spans two chunks), picked by selects over
                // compile-time indices (blocks past nout fall back to the chunk's
                // first and are never written)
                constexpr int BPC = P >= 16 ? 1 : 16 / P;
                TO* ybase = (TO*)out.p[(16 * oc) / P];
#pragma unroll
                for (int u = 1; u < BPC; ++u) {
                    TO* pu = (TO*)out.p[BPC * oc + u < nout ? BPC * oc + u : BPC * oc];
                    ybase = (ob % BPC == u) ? pu : ybase;
                }
                double old[4] = {0, 0, 0, 0};
                if (16 * oc < accumulate * P) {  // some output block of this chunk is accumulated
                    const double keep = ob < accumulate ? 1.0 : 0.0;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        old[v] = keep * as<double>(ybase[clamp_row(rbase + rq + 4 * v, n) * P + (col < N ? b : 0)]);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = rbase + rq + 4 * v;
                    if (row < n && col < N) ybase[row * P + b] = to_store<TO>(acc[oc][v] + old[v]);
                }
                acc[oc] = typename M::acc{0, 0, 0, 0};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// block combination Y (+)= X C with X = [in_0 .. in_{nin-1}] (n x K, K = nin P)
// and Y = [out_0 .. out_{nout-1}] (n x N, N = nout P), C (K x N) row-major in
// FP64: a tall-skinny product on matrix cores in the arithmetic type TC (FP64,
// or FP32 when inputs and outputs are FP32/BF16 blocks; then the
// coefficients are rounded to FP32).  At N = 64 the product is bound by the
// matrix-core rate, not by memory.  The first `accumulate` output blocks are
// accumulated (Y += X C), the others overwritten.
// The pipeline steps over (16-row wave tile, group of G = 64 / P input
// blocks): the group is read with wide loads (the next step's in flight while
// the current one is multiplied), widened into a wave-private LDS tile of type
// TC and read back as the A operand X[row][k]; B = C[k][j] from LDS, padded
// to NCO chunks of 16 output columns.
// ---------------------------------------------------------------------------
template <class TI, class TO, class TC, int P, int NCO>
__global__ __launch_bounds__(256) void k_combine_mfma(int64_t n, BlockPtrs in, int nin, BlockPtrs out, int nout,
                                                      const double* __restrict__ coef, int accumulate) {
    using M = MX<TC>;
    constexpr int KK = P / 4, G = 64 / P, NPAD = 16 * NCO, XLD = 64;
    using Wd = Wide<TI, P, G>;
    const int N = nout * P, K = nin * P;
    extern __shared__ __align__(16) unsigned char smem[];
    TC* Cs = (TC*)smem;                              // [K][NPAD]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, bl = lane & 15, rq = lane >> 4;
    TC* myX = Cs + (size_t)K * NPAD + wave * 16 * XLD;  // [16][XLD] per wave
    for (int e = threadIdx.x; e < K * NPAD; e += 256) {
        const int k = e / NPAD, j = e % NPAD;
        Cs[e] = j < N ? (TC)coef[(int64_t)k * N + j] : (TC)0;
    }
    __syncthreads();
    const int nch = (nin + G - 1) / G;
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    const int64_t nsteps = (t1 - t0) * nch;
    auto load = [&](u4v* buf, int64_t s) {
        const int64_t tile = t0 + s / nch;
        const int c = (int)(s % nch);
        const TI* qb[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int blk = c * G + g;
            qb[g] = (const TI*)in.p[blk < nin ? blk : 0];
        }
        wide_load<TI, P, G>(buf, qb, tile * MROWS + wave * 16, n, lane);
    };
    typename M::acc acc[NCO];
#pragma unroll
    for (int oc = 0; oc < NCO; ++oc) acc[oc] = typename M::acc{0, 0, 0, 0};
    u4v xn[Wd::NIA];
    if (nsteps > 0) load(xn, 0);
    for (int64_t s = 0; s < nsteps; ++s) {
        wide_to_lds<TC, TI, P, G, XLD>(myX, xn, lane);
        if (s + 1 < nsteps) load(xn, s + 1);
        const int c = (int)(s % nch);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int blk = c * G + g;
            if (blk < nin) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const TC a = myX[qsw<XLD>(bl, g * P + 4 * kk + rq)];
                    const TC* cr = Cs + (blk * P + 4 * kk + rq) * NPAD + bl;
#pragma unroll
                    for (int oc = 0; oc < NCO; ++oc) acc[oc] = M::mma(a, cr[16 * oc], acc[oc]);
                }
            }
        }
        if (c == nch - 1) {
            // D[row][col]: lane l element v holds row rbase + drow(l, v), column 16 oc + l % 16
            const int64_t rbase = (t0 + s / nch) * MROWS + wave * 16;
#pragma unroll
            for (int oc = 0; oc < NCO; ++oc) {
                const int col = 16 * oc + bl;
                const int ob = col / P, b = col % P;
                // output block of this lane's column: one of the 16 / P blocks of the
                // chunk, picked by selects over compile-time indices (blocks past
                // nout fall back to the chunk's first and are never written)
                constexpr int BPC = 16 / P;
                TO* ybase = (TO*)out.p[BPC * oc];
#pragma unroll
                for (int u = 1; u < BPC; ++u) {
                    TO* pu = (TO*)out.p[BPC * oc + u < nout ? BPC * oc + u : BPC * oc];
                    ybase = (ob % BPC == u) ? pu : ybase;
                }
                double old[4] = {0, 0, 0, 0};
                if (16 * oc < accumulate * P) {  // some output block of this chunk is accumulated
                    const double keep = ob < accumulate ? 1.0 : 0.0;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        old[v] = keep * as<double>(ybase[clamp_row(rbase + M::drow(lane, v), n) * P + (col < N ? b : 0)]);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = rbase + M::drow(lane, v);
                    if (row < n && col < N) ybase[row * P + b] = to_store<TO>((double)acc[oc][v] + old[v]);
                }
                acc[oc] = typename M::acc{0, 0, 0, 0};
            }
        }
    }
}

// complex blocks of P / 2 columns with complex coefficients (k_combine_scalar
// with CX), P = 16 or 32 real columns, at most 64 of them in the output
template <int P>
hipError_t launch_combine_cx(hipStream_t st, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                             const double* coef, int accumulate, int nwg) {
    const int nco = (nout * P + 15) / 16;
    const size_t lds = (size_t)nin * P * 16 * nco / 2 * sizeof(double);
    if (nin < 1 || nout < 1 || lds > (size_t)160 * 1024) return hipErrorNotSupported;
#define L(NCO)                                                                                                    \
    {                                                                                                             \
        static std::once_flag fl;                                                                                 \
        std::call_once(fl, [] { allow_lds(k_combine_scalar<double, double, P, NCO, true>); });                    \
        hipLaunchKernelGGL((k_combine_scalar<double, double, P, NCO, true>), dim3(nwg), dim3(256), lds, st, n, in, \
                           nin, out, nout, coef, accumulate);                                                     \
    }
    switch (nco) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorNotSupported;
    }
#undef L
    return hipGetLastError();
}

template <class TI, class TO, int P>
hipError_t launch_combine(hipStream_t st, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                          const double* coef, int accumulate, int nwg) {
    // FP32 arithmetic when neither side is FP64 (basis combinations of the
    // FP32 forms); FP64 otherwise (solution updates, FP64 bases)
    using TC = typename std::conditional<!std::is_same<TI, double>::value && !std::is_same<TO, double>::value, float,
                                         double>::type;
    constexpr bool wide = !std::is_same<TI, double>::value;  // FP64 inputs: scalar-load kernel
    const int nco = (nout * P + 15) / 16;
    const size_t lds = ((size_t)nin * P * 16 * nco + (wide ? 4 * 16 * 64 : 0)) * sizeof(TC);
    if (nin < 1 || nout < 1 || lds > (size_t)160 * 1024) return hipErrorNotSupported;
#define L(NCO)                                                                                                     \
    {                                                                                                              \
        if constexpr (wide) {                                                                                      \
            static std::once_flag fl;                                                                              \
            std::call_once(fl, [] { allow_lds(k_combine_mfma<TI, TO, TC, P, NCO>); });                             \
            hipLaunchKernelGGL((k_combine_mfma<TI, TO, TC, P, NCO>), dim3(nwg), dim3(256), lds, st, n, in, nin, out, \
                               nout, coef, accumulate);                                                             \
        } else {                                                                                                   \
            static std::once_flag fl;                                                                              \
            std::call_once(fl, [] { allow_lds(k_combine_scalar<TI, TO, P, NCO>); });                               \
            hipLaunchKernelGGL((k_combine_scalar<TI, TO, P, NCO>), dim3(nwg), dim3(256), lds, st, n, in, nin, out,   \
                               nout, coef, accumulate);                                                             \
        }                                                                                                          \
    }
    switch (nco) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorNotSupported;
    }
#undef L
    return hipGetLastError();
}

template <class T, class TQ, class TO, int P, bool UPD, bool DOT, bool GRAM, bool NORM>
hipError_t launch_sweep_t(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                          TO* Wout, double* part, const double* Rinv, int nwg, const Ctl* ctl, int step) {
    const int nc = (nq * P + 15) / 16;
#define L(NC)                                                                                                     \
    {                                                                                                             \
        constexpr int NQ = NC * 16 / P, NQA = NQ > 0 ? NQ : 1, QLD = 32 * ((NC + 1) / 2);                         \
        constexpr bool TILE = NQ > 0 && (UPD || DOT);                                                             \
        const size_t lds = std::max((size_t)((UPD ? NQA * P * P : 0) + (TILE ? 4 * 16 * QLD : 0) + 4 * 16 * P) *  \
                                        sizeof(T),                                                                \
                                    (size_t)1024 * sizeof(double));                                               \
        if (lds > (size_t)160 * 1024) return hipErrorNotSupported;                                                \
        static std::once_flag fl;                                                                                 \
        std::call_once(fl, [] { allow_lds(k_sweep_mfma<T, TQ, TO, P, NC, UPD, DOT, GRAM, NORM>); });              \
        hipLaunchKernelGGL((k_sweep_mfma<T, TQ, TO, P, NC, UPD, DOT, GRAM, NORM>), dim3(nwg), dim3(256), lds, st, n, \
                           Win, Q, nq, S, Wout, part, Rinv, ctl, step);                                           \
    }
    if (nq == 0) {
        L(0);
        return hipGetLastError();
    }
    BGCR_MX_NC_DISPATCH(nc, L)
#undef L
    return hipGetLastError();
}

}  // namespace mx

// public entry points (declared in bgcr_internal.h), instantiated per type
// Kernel choice per arithmetic type (measured on the sweeps of a block step):
// with FP32 arithmetic the wide-load sweep (16 bytes per lane and load) is
// 1.1-2.9x faster than the scalar-load kernels for every sweep; the FP64
// sweeps keep the scalar-load kernels, which are as fast at P = 8 (where the
// wide prefetch costs occupancy).
template <class T, class TW, class TQ>
hipError_t mfma_dot(hipStream_t st, int P, int64_t n, const BlockPtrs& W, int nw, const BlockPtrs& Q, int nq,
                    double* part, const Ctl* ctl, int nwg, bool rev) {
    if constexpr (sizeof(T) == 4 && std::is_same<TW, T>::value) {
        if (nw == 1 && P == 8)
            return mx::launch_sweep_t<T, TQ, T, 8, false, true, false, false>(st, n, (const T*)W.p[0], Q, nq, nullptr,
                                                                            (T*)nullptr, part, nullptr, nwg, ctl, -1);
        if (nw == 1 && P == 16)
            return mx::launch_sweep_t<T, TQ, T, 16, false, true, false, false>(st, n, (const T*)W.p[0], Q, nq, nullptr,
                                                                             (T*)nullptr, part, nullptr, nwg, ctl, -1);
    }
    if (P == 8) return mx::launch_dot<T, TW, TQ, 8>(st, n, W, nw, Q, nq, part, nwg, ctl, rev);
    if (P == 16) return mx::launch_dot<T, TW, TQ, 16>(st, n, W, nw, Q, nq, part, nwg, ctl, rev);
    // narrow blocks (P < 8, FP64 or FP32 storage): 16 / P blocks per chunk
    if constexpr (std::is_same<TW, T>::value && std::is_same<TQ, T>::value) {
        if (P == 1) return mx::launch_dot<T, T, T, 1>(st, n, W, nw, Q, nq, part, nwg, ctl, rev);
        if (P == 2) return mx::launch_dot<T, T, T, 2>(st, n, W, nw, Q, nq, part, nwg, ctl, rev);
        if (P == 4) return mx::launch_dot<T, T, T, 4>(st, n, W, nw, Q, nq, part, nwg, ctl, rev);
    }
    return hipErrorNotSupported;
}

template <class T, class TQ>
hipError_t mfma_proj_dot(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                         double* part, const Ctl* ctl, int nwg, bool gram, bool rev) {
    if constexpr (sizeof(T) == 4) {
#define BGCR_SWEEP2(PP)                                                                                             \
    return gram ? mx::launch_sweep_t<T, TQ, T, PP, true, true, true, false>(st, n, Win, Q, nq, S, (T*)nullptr, part, \
                                                                            nullptr, nwg, ctl, -1)                   \
                : mx::launch_sweep_t<T, TQ, T, PP, true, true, false, false>(st, n, Win, Q, nq, S, (T*)nullptr, part, \
                                                                             nullptr, nwg, ctl, -1);
        if (P == 8) BGCR_SWEEP2(8)
        if (P == 16) BGCR_SWEEP2(16)
#undef BGCR_SWEEP2
    }
    if (P == 8) return mx::launch_proj_dot<T, TQ, 8>(st, n, Win, Q, nq, S, part, nwg, ctl, gram, rev);
    if (P == 16) return mx::launch_proj_dot<T, TQ, 16>(st, n, Win, Q, nq, S, part, nwg, ctl, gram, rev);
    if constexpr (std::is_same<TQ, T>::value) {
        if (P == 4) return mx::launch_proj_dot<T, T, 4>(st, n, Win, Q, nq, S, part, nwg, ctl, gram, rev);
    }
    return hipErrorNotSupported;
}

template <class T, class TQ, class TO>
hipError_t mfma_proj_gram(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                          const double* S, TO* Wout, double* part, const Ctl* ctl, int nwg, const double* Rinv,
                          int step, bool rev) {
    if constexpr (sizeof(T) == 4) {
#define BGCR_SWEEP3(PP)                                                                                              \
    return Rinv ? mx::launch_sweep_t<T, TQ, TO, PP, true, false, false, true>(st, n, Win, Q, nq, S, Wout, part, Rinv, \
                                                                              nwg, ctl, step)                        \
                : mx::launch_sweep_t<T, TQ, TO, PP, true, false, true, false>(st, n, Win, Q, nq, S, Wout, part, Rinv, \
                                                                              nwg, ctl, step);
        if (P == 8) BGCR_SWEEP3(8)
        if (P == 16) BGCR_SWEEP3(16)
#undef BGCR_SWEEP3
    }
    if (P == 8) return mx::launch_proj_gram<T, TQ, TO, 8>(st, n, Win, Q, nq, S, Wout, part, Rinv, nwg, ctl, step, rev);
    if (P == 16) return mx::launch_proj_gram<T, TQ, TO, 16>(st, n, Win, Q, nq, S, Wout, part, Rinv, nwg, ctl, step, rev);
    if constexpr (std::is_same<TQ, T>::value && std::is_same<TO, T>::value) {
        if (P == 4) return mx::launch_proj_gram<T, T, T, 4>(st, n, Win, Q, nq, S, Wout, part, Rinv, nwg, ctl, step, rev);
    }
    return hipErrorNotSupported;
}

template <class TI, class TO>
hipError_t mfma_combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                        const double* coef, int accumulate, int nwg) {
    if (P == 8) return mx::launch_combine<TI, TO, 8>(st, n, in, nin, out, nout, coef, accumulate, nwg);
    if (P == 16) return mx::launch_combine<TI, TO, 16>(st, n, in, nin, out, nout, coef, accumulate, nwg);
    // four-column FP64 blocks: the scalar-load kernel (a chunk spans 4 output blocks)
    if constexpr (std::is_same<TI, double>::value) {
        if (P == 4) return mx::launch_combine<TI, TO, 4>(st, n, in, nin, out, nout, coef, accumulate, nwg);
    }
    return hipErrorNotSupported;
}

}  // namespace bgcr
