// Matrix-core (MFMA) versions of the three block-Arnoldi sweeps for block
// sizes P = 8 and 16 with real FP64 or FP32 basis storage.
//
// Every sweep streams n rows of a few tall-skinny n x P blocks; all dense
// contractions run on v_mfma_*_16x16x4 tiles:
//   * block-CGS update  W' = W - Q S : (W')^T = W^T + (-S)^T Q^T, contraction
//     over the q columns of Q (K = 4 columns per instruction);
//   * block dot products S = Q^T W   : S^T = W^T Q, contraction over rows
//     (K = 4 rows per instruction), accumulated for the whole row range of a
//     workgroup;
//   * Gram matrix W''^T W'' in FP64 (also for FP32 storage).
// A wave works on 16 rows at a time; a workgroup of 4 waves on 64-row tiles.
// Operand layouts of a 16x16x4 instruction (lane l):
//   A[i][k] = lane (i = l % 16, k = l / 16), B[k][j] = lane (k = l / 16, j = l % 16)
//   D[i][j]: FP64 lane l element v holds i = l/16 + 4v, j = l % 16;
//            FP32 lane l element v holds i = 4(l/16) + v, j = l % 16.
// Results that feed another contraction in a different layout go through a
// 16 x P transposition buffer in LDS per wave.
#include <mutex>

#include "bgcr_internal.h"

namespace bgcr {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <class T> struct MX;
template <> struct MX<double> {
    using acc = d4v;
    __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int drow(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct MX<float> {
    using acc = f4v;
    __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int l, int v) { return 4 * (l >> 4) + v; }
};

__device__ inline int mx_logical_wg() {
    const int w = blockIdx.x, G = gridDim.x;
    if (G % 8 != 0) return w;
    return (w % 8) * (G / 8) + (w / 8);
}

constexpr int MROWS = 64;  // rows per workgroup tile (4 waves x 16 rows)

// Cross-wave reduction of per-wave MFMA dot accumulators and write of the
// workgroup partial: chunk ch of the accumulators holds S^T[b][c] with
// b = drow(l, v), c = 16 ch + l % 16.  Output part[lw][c P + b].
template <class T, int P, int NCM>
__device__ inline void write_dot_partials(typename MX<T>::acc (&acc)[NCM], int nc16, int q, double* red, double* part,
                                          int lw, int nout) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int ch = 0; ch < NCM; ++ch) {
        if (ch < nc16) {
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(wave * 4 + v) * 64 + lane] = (double)acc[ch][v];
            __syncthreads();
            // thread t -> (v, lane) = (t / 64, t % 64): sum the 4 waves in order
            const int v = t >> 6, l = t & 63;
            const double s = red[(0 * 4 + v) * 64 + l] + red[(1 * 4 + v) * 64 + l] + red[(2 * 4 + v) * 64 + l] +
                             red[(3 * 4 + v) * 64 + l];
            const int b = MX<T>::drow(l, v);
            const int c = ch * 16 + (l & 15);
            if (b < P && c < q) part[(int64_t)lw * nout + (int64_t)c * P + b] = s;
        }
    }
}

// Gram accumulator (FP64 MFMA, D[i][j] = G[i][j]) -> part[lw][i P + j]
template <int P>
__device__ inline void write_gram_partials(d4v g, double* red, double* part, int lw, int nout, int off) {
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

// Q operands of the update for the 16 rows rbase..rbase+15 of up to NQM
// blocks, "CR" layout: value blk*KK + kk holds Q_blk[row = l % 16][4 kk + l / 16].
// Block pointers are wave-uniform (scalar loads).
template <class T, int P, int NQM>
__device__ inline void load_update_operands(T (&qv)[NQM * (P / 4)], const BlockPtrs& Q, int nq, int64_t rbase,
                                            int64_t n, int lane) {
    constexpr int KK = P / 4;
    const int64_t row = rbase + (lane & 15);
    const bool ok = row < n;
#pragma unroll
    for (int blk = 0; blk < NQM; ++blk) {
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            qv[blk * KK + kk] = (T)0;
            if (blk < nq && ok) qv[blk * KK + kk] = ((const T*)Q.p[blk])[row * P + 4 * kk + (lane >> 4)];
        }
    }
}

// D (layout of MX<T>) = W^T + (-S)^T Q^T for 16 rows; Ss holds -S as [c][P]
template <class T, int P, int NQM>
__device__ inline typename MX<T>::acc update_mma(typename MX<T>::acc d, const T (&qv)[NQM * (P / 4)], int nq,
                                                 const T* Ss, int lane) {
    constexpr int KK = P / 4;
#pragma unroll
    for (int blk = 0; blk < NQM; ++blk) {
        if (blk < nq) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const T sv = (lane & 15) < P ? Ss[(blk * P + 4 * kk + (lane >> 4)) * P + (lane & 15)] : (T)0;
                d = MX<T>::mma(sv, qv[blk * KK + kk], d);
            }
        }
    }
    return d;
}

template <class T, int P>
__device__ inline typename MX<T>::acc load_wt(const T* __restrict__ Win, int64_t rbase, int64_t n, int lane) {
    typename MX<T>::acc d;
    const int64_t row = rbase + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int b = MX<T>::drow(lane, v);
        d[v] = (b < P && row < n) ? Win[row * P + b] : (T)0;
    }
    return d;
}

// D-layout tile -> row-major 16 x P in LDS
template <class T, int P>
__device__ inline void d_to_lds(const typename MX<T>::acc& d, T* tr, int lane) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int b = MX<T>::drow(lane, v);
        if (b < P) tr[(lane & 15) * P + b] = d[v];
    }
}

// B operand of the dot for 16-column chunk ch from global memory
template <class T, int P>
__device__ inline T dot_operand(const BlockPtrs& Q, int nq, int ch, int64_t row, int64_t n, int lane) {
    const int cl = lane & 15;
    int blk, a;
    if constexpr (P == 16) {
        blk = ch;
        a = cl;
    } else {
        blk = 2 * ch + (cl >> 3);
        a = cl & 7;
    }
    if (blk >= nq || row >= n) return (T)0;
    const T* qp;
    if constexpr (P == 16) {
        qp = (const T*)Q.p[ch];
    } else {
        const T* p0 = (const T*)Q.p[2 * ch];
        const T* p1 = (const T*)Q.p[2 * ch + 1];
        qp = (cl >> 3) ? p1 : p0;
    }
    return qp[row * P + a];
}

// ---------------------------------------------------------------------------
// sweep 2: W' = W - Q S1 (not stored); partial S2 = Q^T W'.
// The Q operands loaded for the update are written to a per-wave LDS tile
// and read back in the layout of the dot; the next tile's operands are loaded
// while the current tile computes.
// ---------------------------------------------------------------------------
template <class T, int P, int NCM>
__global__ __launch_bounds__(256) void k_proj_dot_mfma(int64_t n, const T* __restrict__ Win, BlockPtrs Q, int nq,
                                                       const double* __restrict__ S, double* __restrict__ part,
                                                       const Ctl* ctl) {
    using M = MX<T>;
    constexpr int NQM = NCM * 16 / P, KK = P / 4, NQV = NQM * KK;
    constexpr int QLD = NCM * 16 + 1;  // padded row stride of the LDS Q tile
    if (ctl && ctl->active == 0) return;
    const int q = nq * P, nc16 = (q + 15) / 16;
    extern __shared__ __align__(16) unsigned char smem[];
    T* Ss = (T*)smem;                        // [NQM*P][P]
    T* Qt = Ss + NQM * P * P;                // [4 waves][16][QLD]
    T* Wt = Qt + 4 * 16 * QLD;               // [4 waves][16][P]
    double* red = (double*)smem;             // reused at the end: 1024 doubles
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nup = S ? nq : 0;
    for (int e = t; e < NQM * P * P; e += 256) Ss[e] = (S && e < q * P) ? (T)(-S[e]) : (T)0;
    typename M::acc acc[NCM];
#pragma unroll
    for (int ch = 0; ch < NCM; ++ch) acc[ch] = typename M::acc{0, 0, 0, 0};
    const int lw = mx_logical_wg();
    const int64_t ntiles = (n + MROWS - 1) / MROWS;
    const int64_t t0 = (int64_t)lw * ntiles / gridDim.x, t1 = (int64_t)(lw + 1) * ntiles / gridDim.x;
    T* myQ = Qt + wave * 16 * QLD;
    T* myW = Wt + wave * 16 * P;
    T qn[NQV];
    typename M::acc wn = typename M::acc{0, 0, 0, 0};
    if (t0 < t1) {
        load_update_operands<T, P, NQM>(qn, Q, nq, t0 * MROWS + wave * 16, n, lane);
        wn = load_wt<T, P>(Win, t0 * MROWS + wave * 16, n, lane);
    }
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t rbase = tile * MROWS + wave * 16;
        T qc[NQV];
#pragma unroll
        for (int e = 0; e < NQV; ++e) qc[e] = qn[e];
        typename M::acc d = wn;
        if (tile + 1 < t1) {
            load_update_operands<T, P, NQM>(qn, Q, nq, rbase + MROWS, n, lane);
            wn = load_wt<T, P>(Win, rbase + MROWS, n, lane);
        }
        d = update_mma<T, P, NQM>(d, qc, nup, Ss, lane);
        d_to_lds<T, P>(d, myW, lane);
#pragma unroll
        for (int blk = 0; blk < NQM; ++blk)
#pragma unroll
            for (int kk = 0; kk < KK; ++kk)
                if (blk < nq) myQ[(lane & 15) * QLD + blk * P + 4 * kk + (lane >> 4)] = qc[blk * KK + kk];
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rl = ks * 4 + (lane >> 4);
            const T wv = ((lane & 15) < P) ? myW[rl * P + (lane & 15)] : (T)0;
#pragma unroll
            for (int ch = 0; ch < NCM; ++ch) {
                if (ch < nc16) {
                    const int c = ch * 16 + (lane & 15);
                    const T qv = c < q ? myQ[rl * QLD + c] : (T)0;
                    acc[ch] = M::mma(wv, qv, acc[ch]);
                }
            }
        }
        __syncthreads();
    }
    write_dot_partials<T, P, NCM>(acc, nc16, q, red, part, lw, q * P);
}

// ---------------------------------------------------------------------------
// sweep 3: W'' = W - Q S stored (optional); partial Gram W''^T W'' (FP64)
// ---------------------------------------------------------------------------
template <class T, int P, int NQM>
__global__ __launch_bounds__(256) void k_proj_gram_mfma(int64_t n, const T* __restrict__ Win, BlockPtrs Q, int nq,
                                                        const double* __restrict__ S, T* __restrict__ Wout,
                                                        double* __restrict__ part, const Ctl* ctl) {
    using M = MX<T>;
    constexpr int KK = P / 4, NQV = NQM * KK;
    if (ctl && ctl->active == 0) return;
    const int q = nq * P;
    extern __shared__ __align__(16) unsigned char smem[];
    T* Ss = (T*)smem;                  // [NQM*P][P]
    T* tr = Ss + NQM * P * P;          // [4 waves][16][P]
    double* red = (double*)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int e = t; e < NQM * P * P; e += 256) Ss[e] = (e < q * P) ? (T)(-S[e]) : (T)0;
    d4v gacc = {0, 0, 0, 0};
    const int lw = mx_logical_wg();
    const int64_t ntiles = (n + MROWS - 1) / MROWS;
    const int64_t t0 = (int64_t)lw * ntiles / gridDim.x, t1 = (int64_t)(lw + 1) * ntiles / gridDim.x;
    T* mytr = tr + wave * 16 * P;
    constexpr int NQA = NQV > 0 ? NQM : 1;  // register array size (one dummy block when there is no update)
    T qn[NQA * KK];
    typename M::acc wn = typename M::acc{0, 0, 0, 0};
    if (t0 < t1) {
        if constexpr (NQV > 0) load_update_operands<T, P, NQA>(qn, Q, nq, t0 * MROWS + wave * 16, n, lane);
        wn = load_wt<T, P>(Win, t0 * MROWS + wave * 16, n, lane);
    }
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t rbase = tile * MROWS + wave * 16;
        typename M::acc d = wn;
        if constexpr (NQV > 0) {
            T qc[NQA * KK];
#pragma unroll
            for (int e = 0; e < NQA * KK; ++e) qc[e] = qn[e];
            if (tile + 1 < t1) load_update_operands<T, P, NQA>(qn, Q, nq, rbase + MROWS, n, lane);
            d = update_mma<T, P, NQA>(d, qc, nq, Ss, lane);
        }
        if (tile + 1 < t1) wn = load_wt<T, P>(Win, rbase + MROWS, n, lane);
        const int64_t row = rbase + (lane & 15);
        if (Wout && row < n) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = M::drow(lane, v);
                if (b < P) Wout[row * P + b] = d[v];
            }
        }
        d_to_lds<T, P>(d, mytr, lane);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rl = ks * 4 + (lane >> 4);
            const double wv = ((lane & 15) < P) ? (double)mytr[rl * P + (lane & 15)] : 0.0;
            gacc = MX<double>::mma(wv, wv, gacc);
        }
        __syncthreads();
    }
    write_gram_partials<P>(gacc, red, part, lw, P * P, 0);
}

// ---------------------------------------------------------------------------
// sweep 1: W = (A Vin) Rinv, V_j = Vin Rinv (own rows, stored), partial
// [Q_0..Q_{nq-1}, V_j]^T W.  Row pointers of tile t+2 and the column
// indices/values of tile t+1 are loaded while tile t is gathered and computed.
// ---------------------------------------------------------------------------
template <class T, int P, int NCM>
__global__ __launch_bounds__(256) void k_spmm_dot_mfma(int64_t n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const T* __restrict__ av,
                                                       const T* __restrict__ Vin, const double* __restrict__ Rinv,
                                                       T* __restrict__ Vout, T* __restrict__ Wout, BlockPtrs Q,
                                                       int nq, double* __restrict__ part, const Ctl* ctl) {
    using M = MX<T>;
    constexpr int U = P / 4;
    constexpr int NZ = 8;  // nonzeros per row handled by the pipelined path
    if (ctl && ctl->active == 0) return;
    const int q = (nq + 1) * P, nc16 = (q + 15) / 16;
    extern __shared__ __align__(16) unsigned char smem[];
    T* trw = (T*)smem;               // [4][16][P]  W tile
    T* trv = trw + 4 * 16 * P;       // [4][16][P]  V_j tile (self block of Q)
    double* red = (double*)smem;     // reused at the end (1024 doubles = 8 KB)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    T rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int a = 4 * u + (lane >> 4), b = lane & 15;
        rv[u] = (b < P) ? (T)(Rinv ? Rinv[a * P + b] : (a == b ? 1.0 : 0.0)) : (T)0;
    }
    typename M::acc acc[NCM];
#pragma unroll
    for (int ch = 0; ch < NCM; ++ch) acc[ch] = typename M::acc{0, 0, 0, 0};
    const int lw = mx_logical_wg();
    const int64_t ntiles = (n + MROWS - 1) / MROWS;
    const int64_t t0 = (int64_t)lw * ntiles / gridDim.x, t1 = (int64_t)(lw + 1) * ntiles / gridDim.x;
    T* mw = trw + wave * 16 * P;
    T* mv = trv + wave * 16 * P;
    auto rowof = [&](int64_t tile) { return tile * MROWS + wave * 16 + (lane & 15); };
    // pipeline registers: row extents for tile+1 (ra), indices/values for tile (cn, vn)
    int rs_n = 0, re_n = 0;
    int cn[NZ];
    T vn[NZ];
    auto load_extent = [&](int64_t tile, int& rs, int& re) {
        const int64_t r = rowof(tile);
        rs = re = 0;
        if (tile < t1 && r < n) {
            rs = rp[r];
            re = rp[r + 1];
        }
    };
    auto load_nz = [&](int rs, int re, int (&c)[NZ], T (&v)[NZ]) {
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int kk = rs + u;
            c[u] = kk < re ? ci[kk] : -1;
            v[u] = kk < re ? av[kk] : (T)0;
        }
    };
    int rs_c = 0, re_c = 0;
    if (t0 < t1) {
        load_extent(t0, rs_c, re_c);
        load_nz(rs_c, re_c, cn, vn);
        load_extent(t0 + 1, rs_n, re_n);
    }
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t rbase = tile * MROWS + wave * 16;
        const int64_t row = rbase + (lane & 15);
        const bool ok = row < n;
        int cc[NZ];
        T vc[NZ];
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            cc[u] = cn[u];
            vc[u] = vn[u];
        }
        const int rs = rs_c, re = re_c;
        // gathers of this tile and the dot operands of the earlier Q blocks
        T g[NZ][U], vin[U];
#pragma unroll
        for (int u = 0; u < NZ; ++u)
#pragma unroll
            for (int uu = 0; uu < U; ++uu)
                g[u][uu] = cc[u] >= 0 ? Vin[(int64_t)cc[u] * P + 4 * uu + (lane >> 4)] : (T)0;
#pragma unroll
        for (int u = 0; u < U; ++u) vin[u] = ok ? Vin[row * P + 4 * u + (lane >> 4)] : (T)0;
        T qd[4][NCM];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int ch = 0; ch < NCM; ++ch)
                qd[ks][ch] = ch < nc16 ? dot_operand<T, P>(Q, nq, ch, rbase + ks * 4 + (lane >> 4), n, lane) : (T)0;
        // prefetch: indices of tile+1, row extents of tile+2
        rs_c = rs_n;
        re_c = re_n;
        load_nz(rs_c, re_c, cn, vn);
        load_extent(tile + 2, rs_n, re_n);
        T raw[U];
#pragma unroll
        for (int uu = 0; uu < U; ++uu) raw[uu] = (T)0;
#pragma unroll
        for (int u = 0; u < NZ; ++u)
#pragma unroll
            for (int uu = 0; uu < U; ++uu) raw[uu] += vc[u] * g[u][uu];
        for (int kk = rs + NZ; kk < re; ++kk) {  // rows with more than NZ nonzeros
            const T val = av[kk];
            const int64_t col = ci[kk];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) raw[uu] += val * Vin[col * P + 4 * uu + (lane >> 4)];
        }
        typename M::acc dw = typename M::acc{0, 0, 0, 0}, dv = typename M::acc{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dw = M::mma(rv[u], raw[u], dw);
            dv = M::mma(rv[u], vin[u], dv);
        }
        if (ok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = M::drow(lane, v);
                if (b < P) {
                    Wout[row * P + b] = dw[v];
                    Vout[row * P + b] = dv[v];
                }
            }
        }
        d_to_lds<T, P>(dw, mw, lane);
        d_to_lds<T, P>(dv, mv, lane);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int rl = ks * 4 + (lane >> 4);
            const int64_t r2 = rbase + rl;
            const T wv = ((lane & 15) < P) ? mw[rl * P + (lane & 15)] : (T)0;
#pragma unroll
            for (int ch = 0; ch < NCM; ++ch) {
                if (ch < nc16) {
                    const int c = ch * 16 + (lane & 15);
                    T qv = qd[ks][ch];
                    if (c >= nq * P && c < q && r2 < n) qv = mv[rl * P + (c - nq * P)];
                    acc[ch] = M::mma(wv, qv, acc[ch]);
                }
            }
        }
        __syncthreads();
    }
    write_dot_partials<T, P, NCM>(acc, nc16, q, red, part, lw, q * P);
}

// ---------------------------------------------------------------------------
// launchers: return hipErrorNotSupported when the shape has no MFMA variant
// ---------------------------------------------------------------------------
template <class F>
static void mx_allow_lds(F* f) {
    (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

#define MX_NCM_DISPATCH(nc16, MACRO)            \
    if (nc16 <= 4) {                            \
        MACRO(4);                               \
    } else if (nc16 <= 8) {                     \
        MACRO(8);                               \
    } else if (nc16 <= 12) {                    \
        MACRO(12);                              \
    } else if (nc16 <= 16) {                    \
        MACRO(16);                              \
    } else {                                    \
        return hipErrorNotSupported;            \
    }

template <class T, int P>
static hipError_t launch_proj_dot(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                                  const double* S, double* part, int nwg, const Ctl* ctl) {
    const int q = nq * P, nc16 = (q + 15) / 16;
#define L(NC)                                                                                                \
    {                                                                                                        \
        const size_t lds = std::max((size_t)((NC * 16 / P) * P * P + 4 * 16 * (NC * 16 + 1) + 4 * 16 * P) *  \
                                        sizeof(T),                                                           \
                                    (size_t)1024 * sizeof(double));                                          \
        static std::once_flag fl;                                                                            \
        std::call_once(fl, [] { mx_allow_lds(k_proj_dot_mfma<T, P, NC>); });                                 \
        hipLaunchKernelGGL((k_proj_dot_mfma<T, P, NC>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S,    \
                           part, ctl);                                                                       \
    }
    MX_NCM_DISPATCH(nc16, L)
#undef L
    return hipGetLastError();
}

template <class T, int P>
static hipError_t launch_proj_gram(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                                   const double* S, T* Wout, double* part, int nwg, const Ctl* ctl) {
    const int q = nq * P, nc16 = (q + 15) / 16;
    if (nq == 0) {
        const size_t lds = std::max((size_t)(4 * 16 * P) * sizeof(T), (size_t)1024 * sizeof(double));
        hipLaunchKernelGGL((k_proj_gram_mfma<T, P, 0>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S, Wout, part,
                           ctl);
        return hipGetLastError();
    }
#define L(NC)                                                                                                \
    {                                                                                                        \
        const size_t lds = std::max((size_t)((NC * 16 / P) * P * P + 4 * 16 * P) * sizeof(T),              \
                                    (size_t)1024 * sizeof(double));                                          \
        hipLaunchKernelGGL((k_proj_gram_mfma<T, P, NC * 16 / P>), dim3(nwg), dim3(256), lds, st, n, Win, Q,  \
                           nq, S, Wout, part, ctl);                                                          \
    }
    MX_NCM_DISPATCH(nc16, L)
#undef L
    return hipGetLastError();
}

template <class T, int P>
static hipError_t launch_spmm_dot(hipStream_t st, int64_t n, const int* rp, const int* ci, const T* av,
                                  const T* Vin, const double* Rinv, T* Vout, T* Wout, const BlockPtrs& Q, int nq,
                                  double* part, int nwg, const Ctl* ctl) {
    const int q = (nq + 1) * P, nc16 = (q + 15) / 16;
    const size_t lds = std::max((size_t)(2 * 4 * 16 * P) * sizeof(T), (size_t)1024 * sizeof(double));
#define L(NC)                                                                                                   \
    {                                                                                                           \
        hipLaunchKernelGGL((k_spmm_dot_mfma<T, P, NC>), dim3(nwg), dim3(256), lds, st, n, rp, ci, av, Vin, Rinv, \
                           Vout, Wout, Q, nq, part, ctl);                                                       \
    }
    MX_NCM_DISPATCH(nc16, L)
#undef L
    return hipGetLastError();
}

// out = I - M (P x P): turns a right multiplication W M into the update
// W - W (I - M) of the sweep kernels
__global__ void k_i_minus(const double* __restrict__ M, double* __restrict__ out, int P) {
    const int e = threadIdx.x;
    if (e < P * P) out[e] = ((e / P) == (e % P) ? 1.0 : 0.0) - M[e];
}

hipError_t i_minus(hipStream_t st, const double* M, double* out, int P) {
    hipLaunchKernelGGL(k_i_minus, dim3(1), dim3(256), 0, st, M, out, P);
    return hipGetLastError();
}

int mfma_nwg(int64_t n) {
    const int64_t tiles = (n + MROWS - 1) / MROWS;
    int64_t g = tiles < NWG_MAX ? tiles : NWG_MAX;
    if (g >= 8) g -= g % 8;
    return (int)(g < 1 ? 1 : g);
}

template <class T>
hipError_t mfma_proj_dot(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                         double* part, const Ctl* ctl, int nwg) {
    if (P == 8) return launch_proj_dot<T, 8>(st, n, Win, Q, nq, S, part, nwg, ctl);
    if (P == 16) return launch_proj_dot<T, 16>(st, n, Win, Q, nq, S, part, nwg, ctl);
    return hipErrorNotSupported;
}

template <class T>
hipError_t mfma_proj_gram(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                          const double* S, T* Wout, double* part, const Ctl* ctl, int nwg) {
    if (P == 8) return launch_proj_gram<T, 8>(st, n, Win, Q, nq, S, Wout, part, nwg, ctl);
    if (P == 16) return launch_proj_gram<T, 16>(st, n, Win, Q, nq, S, Wout, part, nwg, ctl);
    return hipErrorNotSupported;
}

template <class T>
hipError_t mfma_spmm_dot(hipStream_t st, int P, int64_t n, const int* rp, const int* ci, const T* av, const T* Vin,
                         const double* Rinv, T* Vout, T* Wout, const BlockPtrs& Q, int nq, double* part,
                         const Ctl* ctl, int nwg) {
    if (P == 8) return launch_spmm_dot<T, 8>(st, n, rp, ci, av, Vin, Rinv, Vout, Wout, Q, nq, part, nwg, ctl);
    if (P == 16) return launch_spmm_dot<T, 16>(st, n, rp, ci, av, Vin, Rinv, Vout, Wout, Q, nq, part, nwg, ctl);
    return hipErrorNotSupported;
}

template hipError_t mfma_proj_dot<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                          const double*, double*, const Ctl*, int);
template hipError_t mfma_proj_dot<float>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                         const double*, double*, const Ctl*, int);
template hipError_t mfma_proj_gram<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                           const double*, double*, double*, const Ctl*, int);
template hipError_t mfma_proj_gram<float>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                          const double*, float*, double*, const Ctl*, int);
template hipError_t mfma_spmm_dot<double>(hipStream_t, int, int64_t, const int*, const int*, const double*,
                                          const double*, const double*, double*, double*, const BlockPtrs&, int,
                                          double*, const Ctl*, int);
template hipError_t mfma_spmm_dot<float>(hipStream_t, int, int64_t, const int*, const int*, const float*,
                                         const float*, const double*, float*, float*, const BlockPtrs&, int, double*,
                                         const Ctl*, int);

}  // namespace bgcr
