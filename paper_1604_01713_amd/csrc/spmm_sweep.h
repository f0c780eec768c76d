// Sweep 1 of a block Arnoldi step on the GPU: W = (A Vin) Rinv and
// V_j = Vin Rinv for a CSR matrix A and row-major n x P blocks.
//
// A lane owns C consecutive columns of one row (16 bytes; LPR = P / C lanes
// per row), so every gather of a neighbour row is one 16-byte load per lane
// and one load instruction of a wave reads a contiguous span of the block.  Nonzeros are taken in batches of NB; index loads are clamped
// into the arrays and padding entries are cancelled by a 0/1 factor (no
// select of a loaded value, which the compiler would turn into a branch that
// waits for the load).  The P x P product with Rinv reads Rinv from LDS
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

// C consecutive values of a row, as 16-byte vector loads/stores when the
// lane's slice is a whole number of 16-byte words (blocks are allocated
// 256-byte aligned and a row of P values starts on a 16-byte boundary then)
typedef double vd2 __attribute__((ext_vector_type(2)));
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

template <class T, int P, int C, bool PIPE>
__global__ __launch_bounds__(256) void k_spmm_rinv(int64_t n, int64_t nnz, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ av,
                                                   const T* __restrict__ Vin, const acc_t<T>* __restrict__ Rinv,
                                                   T* __restrict__ Vout, T* __restrict__ Wout, const Ctl* ctl) {
    using A = acc_t<T>;
    using R = typename std::conditional<std::is_same<T, zd>::value, double, T>::type;  // real scalar of T
    static_assert(P % C == 0, "columns per lane must divide P");
    constexpr int LPR = P / C, ROWS = 256 / LPR, NB = 8;
    if (ctl && ctl->active == 0) return;
    __shared__ A Rs[P * P];
    const int t = threadIdx.x, r = t / LPR, part = t % LPR, c0 = part * C;
    const int lead = (t & 63) - part;  // lane holding columns 0..C-1 of this row
    for (int e = t; e < P * P; e += 256) Rs[e] = Rinv ? Rinv[e] : (e / P == e % P ? A{1.0} : A{});
    __syncthreads();
    // Each XCD owns a contiguous slice of tiles; inside it the workgroups take
    // tiles round-robin, so the resident workgroups of an XCD sweep one compact
    // window and the stencil neighbours of that window stay in its L2.
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    const int G = gridDim.x;
    int64_t first, step, end;
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
    const int64_t nzl = nnz - 1;
    auto load_nz = [&](int kb, int (&cols)[NB], T (&vals)[NB]) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int64_t kk = (int64_t)kb + u < nzl ? (int64_t)kb + u : nzl;
            cols[u] = ci[kk];
            vals[u] = av[kk];
        }
    };
    // raw += sum over one batch of nonzeros (entries at or past e cancelled)
    auto accumulate = [&](T (&raw)[C], const int (&cols)[NB], const T (&vals)[NB], int kb, int e) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            T g[C];
            load_cols<T, C, P>(g, Vin + (int64_t)cols[u] * P + c0);
            const T a = mscale(vals[u], (R)(kb + u < e ? 1 : 0));
#pragma unroll
            for (int j = 0; j < C; ++j) raw[j] += a * g[j];
        }
    };
    // W = raw Rinv, V = vb Rinv for this lane's columns c0 .. c0 + C - 1
    auto finish = [&](const T (&raw)[C], const T (&vb)[C], int64_t row) {
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
            store_cols<T, C, P>(Wout + row * P + c0, wo);
            store_cols<T, C, P>(Vout + row * P + c0, vo);
        }
    };
    if (nnz <= 0) {  // A = 0: W = 0, V_j = Vin Rinv
        for (int64_t tile = first; tile < end; tile += step) {
            const int64_t row = tile * ROWS + r;
            T raw[C], vb[C];
#pragma unroll
            for (int j = 0; j < C; ++j) raw[j] = tzero<T>();
            load_cols<T, C, P>(vb, Vin + clamp_row(row, n) * P + c0);
            finish(raw, vb, row);
        }
        return;
    }
    if constexpr (!PIPE) {
        for (int64_t tile = first; tile < end; tile += step) {
            const int64_t row = tile * ROWS + r;
            const int64_t rowc = clamp_row(row, n);
            T raw[C], vb[C];
#pragma unroll
            for (int j = 0; j < C; ++j) raw[j] = tzero<T>();
            load_cols<T, C, P>(vb, Vin + rowc * P + c0);
            const int beg = rp[rowc], e = rp[rowc + 1];
            for (int kb = beg; kb < e; kb += NB) {
                int cols[NB];
                T vals[NB];
                load_nz(kb, cols, vals);
                accumulate(raw, cols, vals, kb, e);
            }
            finish(raw, vb, row);
        }
    } else {
        // software pipeline over the tiles: gathers of tile t, nonzeros of
        // tile t+1 and row pointers of tile t+2 in flight together
        if (first >= end) return;
        int beg0, e0, beg1 = 0, e1 = 0;
        {
            const int64_t rc0 = clamp_row(first * ROWS + r, n);
            beg0 = rp[rc0];
            e0 = rp[rc0 + 1];
        }
        if (first + step < end) {
            const int64_t rc1 = clamp_row((first + step) * ROWS + r, n);
            beg1 = rp[rc1];
            e1 = rp[rc1 + 1];
        }
        int cols[NB];
        T vals[NB];
        load_nz(beg0, cols, vals);
        for (int64_t tile = first; tile < end; tile += step) {
            const int64_t row = tile * ROWS + r;
            T vb[C];
            load_cols<T, C, P>(vb, Vin + clamp_row(row, n) * P + c0);
            T g[NB][C];
#pragma unroll
            for (int u = 0; u < NB; ++u) load_cols<T, C, P>(g[u], Vin + (int64_t)cols[u] * P + c0);
            const int cb = beg0, ce = e0;
            T cv[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) cv[u] = vals[u];
            if (tile + step < end) {
                load_nz(beg1, cols, vals);
                beg0 = beg1;
                e0 = e1;
                if (tile + 2 * step < end) {
                    const int64_t rc2 = clamp_row((tile + 2 * step) * ROWS + r, n);
                    beg1 = rp[rc2];
                    e1 = rp[rc2 + 1];
                }
            }
            T raw[C];
#pragma unroll
            for (int j = 0; j < C; ++j) raw[j] = tzero<T>();
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const T a = mscale(cv[u], (R)(cb + u < ce ? 1 : 0));
#pragma unroll
                for (int j = 0; j < C; ++j) raw[j] += a * g[u][j];
            }
            for (int kb = cb + NB; kb < ce; kb += NB) {  // rows with more than NB nonzeros
                int xc[NB];
                T xv[NB];
                load_nz(kb, xc, xv);
                accumulate(raw, xc, xv, kb, ce);
            }
            finish(raw, vb, row);
        }
    }
}

// columns per lane: 16 bytes, so that a load instruction of a wave reads one
// contiguous span of the block (measured fastest on the 7-point stencil:
// about 1.5x the throughput of one lane per column or per row)
template <class T, int P>
constexpr int spmm_cols() {
    return P < (int)(16 / sizeof(T)) ? P : (int)(16 / sizeof(T));
}

template <class T, int P, int C, bool PIPE>
hipError_t launch_spmm_rinv(hipStream_t st, int64_t n, int64_t nnz, const int* rp, const int* ci, const T* av,
                            const T* Vin, const acc_t<T>* Rinv, T* Vout, T* Wout, const Ctl* ctl, int max_wg) {
    constexpr int ROWS = 256 / (P / C);
    const int64_t tiles = (n + ROWS - 1) / ROWS;
    int64_t g = tiles < max_wg ? tiles : max_wg;
    if (g >= 8) g -= g % 8;
    const int nwg = (int)(g < 1 ? 1 : g);
    hipLaunchKernelGGL((k_spmm_rinv<T, P, C, PIPE>), dim3(nwg), dim3(256), 0, st, n, nnz, rp, ci, av, Vin, Rinv, Vout,
                       Wout, ctl);
    return hipGetLastError();
}

}  // namespace sp
}  // namespace bgcr
