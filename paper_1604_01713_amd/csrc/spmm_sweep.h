// Sweep 1 of a block Arnoldi step on the GPU: W = (A Vin) Rinv and
// V_j = Vin Rinv for a CSR matrix A and row-major n x P blocks, or W = A Vin
// alone when Vin is already normalised (no Rinv and no V_j output).
//
// A lane owns C consecutive columns of one row (16 bytes; LPR = P / C lanes
// per row), so every gather of a neighbour row is one 16-byte load per lane
// and one load instruction of a wave reads a contiguous span of the block.
// With 4 lanes per row, each lane loads a quarter of a batch's column indices
// and values and the batch is assembled by quad broadcasts.  The matrix is
// read once per sweep and is loaded with the non-temporal hint.  Nonzeros
// are taken in batches of NB; index loads are clamped into the arrays and
// padding entries are cancelled by a 0/1 factor (no select of a loaded value,
// which the compiler would turn into a branch that waits for the load).  The P x P product with Rinv reads Rinv from LDS
// (broadcast) and takes the other lanes' columns of the row by wave shuffles.
#pragma once

#include <type_traits>

#include "bgcr_internal.h"

namespace bgcr {
namespace sp {

__device__ inline float mscale(float x, float m) { return x * m; }
__device__ inline double mscale(double x, double m) { return x * m; }
__device__ inline zd mscale(zd x, double m) { return {x.x * m, x.y * m}; }
__device__ inline float shfl_t(float v, int src) { return __shfl(v, src); }
__device__ inline double shfl_t(double v, int src) { return __shfl(v, src); }
__device__ inline zd shfl_t(zd v, int src) { return {__shfl(v.x, src), __shfl(v.y, src)}; }
__device__ inline int64_t clamp_row(int64_t row, int64_t n) { return row < n ? row : n - 1; }

template <class T> __device__ inline T tzero() { return T{}; }

typedef double vd2 __attribute__((ext_vector_type(2)));
// load with the non-temporal hint (data read once)
__device__ inline float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ inline double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
__device__ inline zd ld_nt(const zd* p) {
    const vd2 v = __builtin_nontemporal_load((const vd2*)p);
    return {v[0], v[1]};
}

// value of lane q of each group of 4 lanes (DPP quad_perm broadcast)
template <int Q>
__device__ inline int quad_bcast_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, Q * 0x55, 0xF, 0xF, false);
}
__device__ inline int quad_bcast(int v, int q) {
    switch (q) {
        case 0: return quad_bcast_i<0>(v);
        case 1: return quad_bcast_i<1>(v);
        case 2: return quad_bcast_i<2>(v);
        default: return quad_bcast_i<3>(v);
    }
}
__device__ inline double quad_bcast(double v, int q) {
    const long long b = __double_as_longlong(v);
    const int lo = quad_bcast((int)(b & 0xffffffffll), q), hi = quad_bcast((int)(b >> 32), q);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float quad_bcast(float v, int q) { return __int_as_float(quad_bcast(__float_as_int(v), q)); }
__device__ inline zd quad_bcast(zd v, int q) { return {quad_bcast(v.x, q), quad_bcast(v.y, q)}; }

// C consecutive values of a row, as 16-byte vector loads/stores when the
// lane's slice is a whole number of 16-byte words (blocks are allocated
// 256-byte aligned and a row of P values starts on a 16-byte boundary then)
typedef float vf4 __attribute__((ext_vector_type(4)));

template <class T, int C, int P>
constexpr bool vec16() {
    return (C * sizeof(T)) % 16 == 0 && (P * sizeof(T)) % 16 == 0;
}

template <class T, int C, int P>
__device__ inline void load_cols(T (&v)[C], const T* __restrict__ p) {
    if constexpr (vec16<T, C, P>() && std::is_same<T, float>::value) {
#pragma unroll
        for (int k = 0; k < C / 4; ++k) {
            const vf4 x = *(const vf4*)(p + 4 * k);
            v[4 * k] = x[0];
            v[4 * k + 1] = x[1];
            v[4 * k + 2] = x[2];
            v[4 * k + 3] = x[3];
        }
    } else if constexpr (vec16<T, C, P>()) {
        const double* q = (const double*)p;
        double* d = (double*)v;
#pragma unroll
        for (int k = 0; k < (int)(C * sizeof(T) / 16); ++k) {
            const vd2 x = *(const vd2*)(q + 2 * k);
            d[2 * k] = x[0];
            d[2 * k + 1] = x[1];
        }
    } else {
#pragma unroll
        for (int j = 0; j < C; ++j) v[j] = p[j];
    }
}

template <class T, int C, int P>
__device__ inline void store_cols(T* __restrict__ p, const T (&v)[C]) {
    if constexpr (vec16<T, C, P>() && std::is_same<T, float>::value) {
#pragma unroll
        for (int k = 0; k < C / 4; ++k) *(vf4*)(p + 4 * k) = vf4{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
    } else if constexpr (vec16<T, C, P>()) {
        double* q = (double*)p;
        const double* d = (const double*)v;
#pragma unroll
        for (int k = 0; k < (int)(C * sizeof(T) / 16); ++k) *(vd2*)(q + 2 * k) = vd2{d[2 * k], d[2 * k + 1]};
    } else {
#pragma unroll
        for (int j = 0; j < C; ++j) p[j] = v[j];
    }
}

// SCALE false: W = A Vin only (Vin already normalised; no Rinv, no V_j store)
// C consecutive BF16 values of a row (C = 2 or 4: one 4- or 8-byte load or
// store) converted from / to the arithmetic type T
typedef unsigned int vu2 __attribute__((ext_vector_type(2)));
template <class T, int C>
__device__ inline void load_cols_bf16(T (&v)[C], const bf16* __restrict__ p) {
    static_assert(C == 2 || C == 4, "BF16 rows are gathered 2 or 4 columns per lane");
    unsigned w[C / 2];
    if constexpr (C == 4) {
        const vu2 x = *(const vu2*)p;
        w[0] = x[0];
        w[1] = x[1];
    } else {
        w[0] = *(const unsigned*)p;
    }
#pragma unroll
    for (int k = 0; k < C / 2; ++k) {
        v[2 * k] = (T)__uint_as_float(w[k] << 16);
        v[2 * k + 1] = (T)__uint_as_float(w[k] & 0xffff0000u);
    }
}
template <class T, int C>
__device__ inline void store_cols_bf16(bf16* __restrict__ p, const T (&v)[C]) {
    static_assert(C == 2 || C == 4, "BF16 rows are stored 2 or 4 columns per lane");
    unsigned w[C / 2];
#pragma unroll
    for (int k = 0; k < C / 2; ++k)
        w[k] = (unsigned)float_to_bf16((float)v[2 * k]).u | ((unsigned)float_to_bf16((float)v[2 * k + 1]).u << 16);
    if constexpr (C == 4)
        *(vu2*)p = vu2{w[0], w[1]};
    else
        *(unsigned*)p = w[0];
}
// load / store C columns held as TS (T itself or BF16)
template <class T, class TS, int C, int P>
__device__ inline void load_as(T (&v)[C], const TS* __restrict__ p) {
    if constexpr (std::is_same<TS, bf16>::value)
        load_cols_bf16<T, C>(v, p);
    else
        load_cols<T, C, P>(v, p);
}
template <class T, class TS, int C, int P>
__device__ inline void store_as(TS* __restrict__ p, const T (&v)[C]) {
    if constexpr (std::is_same<TS, bf16>::value)
        store_cols_bf16<T, C>(p, v);
    else
        store_cols<T, C, P>(p, v);
}

// Tiles of ROWS rows taken by this workgroup: each XCD owns a contiguous
// slice of tiles and inside it the workgroups take tiles round-robin, so the
// resident workgroups of an XCD sweep one compact window and the stencil
// neighbours of that window stay in its L2.
__device__ inline void xcd_tiles(int64_t ntiles, int64_t& first, int64_t& step, int64_t& end) {
    const int G = gridDim.x;
    if (G % 8 == 0) {
        const int x = blockIdx.x % 8, i = blockIdx.x / 8;
        first = (int64_t)x * ntiles / 8 + i;
        step = G / 8;
        end = (int64_t)(x + 1) * ntiles / 8;
    } else {
        first = blockIdx.x;
        step = G;
        end = ntiles;
    }
}

// raw[r][0..C-1] = sum over row rowc[r] of A of a_rk Vin[k][c0 .. c0 + C - 1]
// for RR rows at once, their loads issued together (measured: two rows per
// lane are no faster than one on the 7-point stencil; both kernels use one).
// Nonzeros are taken in batches of NB = 8 with indices clamped to nzl =
// nnz - 1 and padding entries cancelled by a 0/1 factor; with SHARE (4 lanes
// per row, `prt` the lane's position) each lane loads 2 entries of a batch
// and the batch is assembled by quad broadcasts.
template <class T, class TI, int P, int C, bool SHARE, int RR>
__device__ inline void row_product(T (&raw)[RR][C], const int* __restrict__ rp, const int* __restrict__ ci,
                                   const T* __restrict__ av, const TI* __restrict__ Vin, const int64_t (&rowc)[RR],
                                   int prt, int c0, int64_t nzl) {
    using R = typename std::conditional<std::is_same<T, zd>::value, double, T>::type;  // real scalar of T
    constexpr int NB = 8;
    int beg[RR], e[RR], len = 0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
        for (int j = 0; j < C; ++j) raw[r][j] = tzero<T>();
        beg[r] = __builtin_nontemporal_load(rp + rowc[r]);
        e[r] = __builtin_nontemporal_load(rp + rowc[r] + 1);
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) len = e[r] - beg[r] > len ? e[r] - beg[r] : len;
    for (int kb0 = 0; kb0 < len; kb0 += NB) {
        int cols[RR][NB];
        T vals[RR][NB];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int kb = beg[r] + kb0;
            if constexpr (SHARE) {
                int mc[2];
                T mv[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t kk = (int64_t)kb + 2 * prt + h < nzl ? (int64_t)kb + 2 * prt + h : nzl;
                    mc[h] = __builtin_nontemporal_load(ci + kk);
                    mv[h] = ld_nt(av + kk);
                }
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    cols[r][u] = quad_bcast(mc[u & 1], u >> 1);
                    vals[r][u] = quad_bcast(mv[u & 1], u >> 1);
                }
            } else {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int64_t kk = (int64_t)kb + u < nzl ? (int64_t)kb + u : nzl;
                    cols[r][u] = __builtin_nontemporal_load(ci + kk);
                    vals[r][u] = ld_nt(av + kk);
                }
            }
        }
        // all gathers of the batch are issued before the first product, so
        // that their latencies overlap
        T g[RR][NB][C];
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int u = 0; u < NB; ++u) load_as<T, TI, C, P>(g[r][u], Vin + (int64_t)cols[r][u] * P + c0);
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const T a = mscale(vals[r][u], (R)(beg[r] + kb0 + u < e[r] ? 1 : 0));
#pragma unroll
                for (int j = 0; j < C; ++j) raw[r][j] += a * g[r][u][j];
            }
    }
}

template <class T, class TI, class TV, class TW, int P, int C, bool SHARE, bool SCALE>
__global__ __launch_bounds__(256) void k_spmm_rinv(int64_t n, int64_t nnz, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ av,
                                                   const TI* __restrict__ Vin, const acc_t<T>* __restrict__ Rinv,
                                                   TV* __restrict__ Vout, TW* __restrict__ Wout, const Ctl* ctl) {
    using A = acc_t<T>;
    static_assert(P % C == 0, "columns per lane must divide P");
    static_assert(!SHARE || P / C == 4, "shared nonzero loads need 4 lanes per row");
    constexpr int LPR = P / C, ROWS = 256 / LPR;
    if (ctl && ctl->active == 0) return;
    __shared__ A Rs[SCALE ? P * P : 1];
    const int t = threadIdx.x, r = t / LPR, part = t % LPR, c0 = part * C;
    const int lead = (t & 63) - part;  // lane holding columns 0..C-1 of this row
    if constexpr (SCALE) {
        for (int e = t; e < P * P; e += 256) Rs[e] = Rinv ? Rinv[e] : (e / P == e % P ? A{1.0} : A{});
        __syncthreads();
    }
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    int64_t first, step, end;
    xcd_tiles(ntiles, first, step, end);
    const int64_t nzl = nnz - 1;
    // W = raw Rinv, V = vb Rinv for this lane's columns c0 .. c0 + C - 1
    auto finish = [&](const T (&raw)[C], const T (&vb)[C], int64_t row) {
        if constexpr (!SCALE) {
            if (row < n) store_as<T, TW, C, P>(Wout + row * P + c0, raw);
            return;
        }
        A w[C], v[C];
#pragma unroll
        for (int j = 0; j < C; ++j) w[j] = v[j] = A{};
#pragma unroll
        for (int q = 0; q < LPR; ++q) {
#pragma unroll
            for (int a = 0; a < C; ++a) {
                const T ra = LPR == 1 ? raw[a] : shfl_t(raw[a], lead + q);
                const T va = LPR == 1 ? vb[a] : shfl_t(vb[a], lead + q);
                const A* rr = Rs + (q * C + a) * P + c0;
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    w[j] += widen(ra) * rr[j];
                    v[j] += widen(va) * rr[j];
                }
            }
        }
        if (row < n) {
            T wo[C], vo[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                wo[j] = narrow<T>(w[j]);
                vo[j] = narrow<T>(v[j]);
            }
            store_as<T, TW, C, P>(Wout + row * P + c0, wo);
            store_as<T, TV, C, P>(Vout + row * P + c0, vo);
        }
    };
    // (with nnz = 0 every row is empty and no index is loaded)
    for (int64_t tile = first; tile < end; tile += step) {
        const int64_t row = tile * ROWS + r;
        const int64_t rowc[1] = {clamp_row(row, n)};
        T raw[1][C], vb[C];
        if constexpr (SCALE) load_as<T, TI, C, P>(vb, Vin + rowc[0] * P + c0);
        row_product<T, TI, P, C, SHARE, 1>(raw, rp, ci, av, Vin, rowc, part, c0, nzl);
        finish(raw[0], vb, row);
    }
}

// R = B - A X in the matrix type (FP64 or complex128) for row-major n x P
// blocks (B with leading dimension ldb), with the lane layout of the block
// SpMM; optional store of R as TR; per-workgroup partial column sums of |r|^2
// and |b|^2 into part[wg][2P] ([P of r][P of b]) in a fixed order.
template <class TA, class TR, int P, int C, bool SHARE>
__global__ __launch_bounds__(256) void k_residual_rows(int64_t n, int64_t nnz, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const TA* __restrict__ av,
                                                       const TA* __restrict__ B, int64_t ldb, const TA* __restrict__ X,
                                                       TR* __restrict__ Rout, double* __restrict__ part) {
    constexpr int LPR = P / C, ROWS = 256 / LPR;
    __shared__ double red[2 * 256 * C];
    const int t = threadIdx.x, r = t / LPR, prt = t % LPR, c0 = prt * C;
    int64_t first, step, end;
    xcd_tiles((n + ROWS - 1) / ROWS, first, step, end);
    const int64_t nzl = nnz - 1;
    double rs[C], bs[C];
#pragma unroll
    for (int j = 0; j < C; ++j) rs[j] = bs[j] = 0.0;
    for (int64_t tile = first; tile < end; tile += step) {
        const int64_t row = tile * ROWS + r;
        const int64_t rowc = clamp_row(row, n);
        TA ax[1][C], bv[C];
        const int64_t rows1[1] = {rowc};
        row_product<TA, TA, P, C, SHARE, 1>(ax, rp, ci, av, X, rows1, prt, c0, nzl);
#pragma unroll
        for (int j = 0; j < C; ++j) bv[j] = B[rowc * ldb + c0 + j];
        const double f = row < n ? 1.0 : 0.0;  // rows past n count nothing
        TR ro[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const TA rv = bv[j] - ax[0][j];
            rs[j] += f * absq(rv);
            bs[j] += f * absq(bv[j]);
            ro[j] = narrow<TR>(rv);
        }
        if (Rout && row < n) store_cols<TR, C, P>(Rout + row * P + c0, ro);
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
        red[t * C + j] = rs[j];
        red[(256 + t) * C + j] = bs[j];
    }
    __syncthreads();
    if (t < 2 * P) {
        const int which = t / P, b = t % P, pr = b / C, j = b % C;
        double a = 0.0;
        for (int rr = 0; rr < ROWS; ++rr) a += red[(which * 256 + rr * LPR + pr) * C + j];
        part[(int64_t)blockIdx.x * 2 * P + t] = a;
    }
}

// Narrow real blocks (P <= 4): S lanes per row, each lane taking every S-th
// nonzero of its row (NB per lane and batch, all P columns), the partial sums
// combined over the S lanes by cross-lane exchanges; the row's first lane
// scales (SCALE: W = raw R^{-1}, V_j = Vin R^{-1}) and stores.  Indices past
// the row are clamped and cancelled by a 0/1 factor.
template <class T, class TI, class TV, class TW, int P, int S, int NB, bool SCALE>
__global__ __launch_bounds__(256) void k_spmm_split(int64_t n, int64_t nnz, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const T* __restrict__ av,
                                                    const TI* __restrict__ Vin, const acc_t<T>* __restrict__ Rinv,
                                                    TV* __restrict__ Vout, TW* __restrict__ Wout, const Ctl* ctl) {
    static_assert(std::is_same<T, double>::value || std::is_same<T, float>::value, "real blocks");
    static_assert(64 % S == 0, "rows must not straddle a wave");
    using A = acc_t<T>;
    constexpr int ROWS = 256 / S;
    if (ctl && ctl->active == 0) return;
    __shared__ A Rs[SCALE ? P * P : 1];
    const int t = threadIdx.x, r = t / S, prt = t % S;
    if constexpr (SCALE) {
        for (int e = t; e < P * P; e += 256) Rs[e] = Rinv ? Rinv[e] : (e / P == e % P ? A{1.0} : A{});
        __syncthreads();
    }
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    int64_t first, step, end;
    xcd_tiles(ntiles, first, step, end);
    const int64_t nzl = nnz - 1;
    for (int64_t tile = first; tile < end; tile += step) {
        const int64_t row = tile * ROWS + r;
        const int64_t rowc = clamp_row(row, n);
        const int beg = __builtin_nontemporal_load(rp + rowc);
        const int e = __builtin_nontemporal_load(rp + rowc + 1);
        T acc[P];
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] = T(0);
        for (int kb = beg; kb < e; kb += S * NB) {
            int cols[NB];
            T vals[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int64_t kk = (int64_t)kb + prt + S * u;
                const int64_t kc = kk < nzl ? kk : nzl;
                cols[u] = __builtin_nontemporal_load(ci + kc);
                vals[u] = ld_nt(av + kc);
            }
            T g[NB][P];
#pragma unroll
            for (int u = 0; u < NB; ++u) load_as<T, TI, P, P>(g[u], Vin + (int64_t)cols[u] * P);
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const T a = mscale(vals[u], (T)((int64_t)kb + prt + S * u < e ? 1 : 0));
#pragma unroll
                for (int j = 0; j < P; ++j) acc[j] += a * g[u][j];
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int off = 1; off < S; off <<= 1) acc[j] += __shfl_xor(acc[j], off, 64);
        if (prt == 0 && row < n) {
            if constexpr (!SCALE) {
                store_as<T, TW, P, P>(Wout + row * P, acc);
            } else {
                T vb[P];
                load_as<T, TI, P, P>(vb, Vin + row * P);
                T wo[P], vo[P];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    A w = A{}, v = A{};
#pragma unroll
                    for (int a = 0; a < P; ++a) {
                        w += widen(acc[a]) * Rs[a * P + j];
                        v += widen(vb[a]) * Rs[a * P + j];
                    }
                    wo[j] = narrow<T>(w);
                    vo[j] = narrow<T>(v);
                }
                store_as<T, TW, P, P>(Wout + row * P, wo);
                store_as<T, TV, P, P>(Vout + row * P, vo);
            }
        }
    }
}

template <class T, class TI, class TV, class TW, int P>
hipError_t launch_spmm_split(hipStream_t st, int64_t n, int64_t nnz, const int* rp, const int* ci, const T* av,
                             const TI* Vin, const acc_t<T>* Rinv, TV* Vout, TW* Wout, const Ctl* ctl, int max_wg) {
    constexpr int S = 4, NB = 2, ROWS = 256 / S;
    const int64_t tiles = (n + ROWS - 1) / ROWS;
    int64_t g = tiles < max_wg ? tiles : max_wg;
    if (g >= 8) g -= g % 8;
    const int nwg = (int)(g < 1 ? 1 : g);
    if (Vout)
        hipLaunchKernelGGL((k_spmm_split<T, TI, TV, TW, P, S, NB, true>), dim3(nwg), dim3(256), 0, st, n, nnz, rp, ci,
                           av, Vin, Rinv, Vout, Wout, ctl);
    else if (Rinv)
        return hipErrorInvalidValue;
    else
        hipLaunchKernelGGL((k_spmm_split<T, TI, TV, TW, P, S, NB, false>), dim3(nwg), dim3(256), 0, st, n, nnz, rp,
                           ci, av, Vin, Rinv, Vout, Wout, ctl);
    return hipGetLastError();
}

// columns per lane: 16 bytes, so that a load instruction of a wave reads one
// contiguous span of the block (measured fastest on the 7-point stencil:
// about 1.5x the throughput of one lane per column or per row).  Complex
// blocks of 8 and 16 columns take 4 lanes per row instead (32 or 64 bytes per
// lane): the row's nonzeros are then shared by quad broadcasts, and the
// R^{-1} product needs a quarter of the cross-lane exchanges of 16 lanes.
template <class T, int P>
constexpr int spmm_cols() {
    if constexpr (std::is_same<T, zd>::value) return P <= 4 ? 1 : P / 4;
    return P < (int)(16 / sizeof(T)) ? P : (int)(16 / sizeof(T));
}

template <class T, class TI, class TV, class TW, int P, int C, bool SHARE>
hipError_t launch_spmm_rinv(hipStream_t st, int64_t n, int64_t nnz, const int* rp, const int* ci, const T* av,
                            const TI* Vin, const acc_t<T>* Rinv, TV* Vout, TW* Wout, const Ctl* ctl, int max_wg) {
    constexpr int ROWS = 256 / (P / C);
    const int64_t tiles = (n + ROWS - 1) / ROWS;
    int64_t g = tiles < max_wg ? tiles : max_wg;
    if (g >= 8) g -= g % 8;
    const int nwg = (int)(g < 1 ? 1 : g);
    if (Vout)
        hipLaunchKernelGGL((k_spmm_rinv<T, TI, TV, TW, P, C, SHARE, true>), dim3(nwg), dim3(256), 0, st, n, nnz, rp, ci, av, Vin,
                           Rinv, Vout, Wout, ctl);
    else if (Rinv)
        return hipErrorInvalidValue;  // a scaled product needs its V_j output
    else
        hipLaunchKernelGGL((k_spmm_rinv<T, TI, TV, TW, P, C, SHARE, false>), dim3(nwg), dim3(256), 0, st, n, nnz, rp, ci, av, Vin,
                           Rinv, Vout, Wout, ctl);
    return hipGetLastError();
}

}  // namespace sp

template <class TA, class TR>
hipError_t residual_rows(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const TA* av,
                         const TA* B, int64_t ldb, const TA* X, TR* Rout, double* part, int nwg) {
#define BGCR_RES_L(PP)                                                                                            \
    {                                                                                                             \
        constexpr int C = sp::spmm_cols<TA, PP>();                                                                \
        hipLaunchKernelGGL((sp::k_residual_rows<TA, TR, PP, C, PP / C == 4>), dim3(nwg), dim3(256), 0, st, n, nnz, \
                           rp, ci, av, B, ldb, X, Rout, part);                                                    \
        return hipGetLastError();                                                                                 \
    }
    switch (P) {
        case 1: BGCR_RES_L(1)
        case 2: BGCR_RES_L(2)
        case 4: BGCR_RES_L(4)
        case 8: BGCR_RES_L(8)
        case 16: BGCR_RES_L(16)
        default: return hipErrorInvalidValue;
    }
#undef BGCR_RES_L
}

template <class T, class TI, class TV, class TW>
hipError_t spmm_block(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const T* av,
                      const TI* Vin, const acc_t<T>* Rinv, TV* Vout, TW* Wout, const Ctl* ctl) {
    // BF16 blocks are gathered 2 or 4 columns per lane: P = 8 and 16 only
    constexpr bool half =
        std::is_same<TI, bf16>::value || std::is_same<TV, bf16>::value || std::is_same<TW, bf16>::value;
#define BGCR_SP_L(PP)                                                                                              \
    return sp::launch_spmm_rinv<T, TI, TV, TW, PP, sp::spmm_cols<T, PP>(), PP / sp::spmm_cols<T, PP>() == 4>(      \
        st, n, nnz, rp, ci, av, Vin, Rinv, Vout, Wout, ctl, 2048);
    if (P == 8) BGCR_SP_L(8)
    if (P == 16) BGCR_SP_L(16)
    if constexpr (!half) {
        // real blocks of up to 4 columns: rows split over 4 lanes
        if constexpr (std::is_same<T, double>::value || std::is_same<T, float>::value) {
            if (P == 1) return sp::launch_spmm_split<T, TI, TV, TW, 1>(st, n, nnz, rp, ci, av, Vin, Rinv, Vout, Wout, ctl, 2048);
            if (P == 2) return sp::launch_spmm_split<T, TI, TV, TW, 2>(st, n, nnz, rp, ci, av, Vin, Rinv, Vout, Wout, ctl, 2048);
            if (P == 4) return sp::launch_spmm_split<T, TI, TV, TW, 4>(st, n, nnz, rp, ci, av, Vin, Rinv, Vout, Wout, ctl, 2048);
        }
        if (P == 1) BGCR_SP_L(1)
        if (P == 2) BGCR_SP_L(2)
        if (P == 4) BGCR_SP_L(4)
    }
#undef BGCR_SP_L
    return hipErrorInvalidValue;
}

}  // namespace bgcr
