// ILU(0) right preconditioning (the incomplete LU factorization the paper
// applies to every system of its convergence experiments, Sections 6.1 and
// 6.2): the numeric factorization and the two triangular solves of
// M^{-1} = U^{-1} L^{-1}, level-scheduled.
//
// The factors share the CSR pattern of A: `lu` holds the strictly lower part
// of L (unit diagonal implied) and the upper part of U, entry for entry where
// A has its nonzeros, with diag[i] the position of (i, i).  Rows are
// processed level by level: a row's level in L is one more than the largest
// level of the rows its strictly lower part refers to (in U the same with the
// strictly upper part), so the rows of one level depend only on earlier
// levels and run in parallel; one launch per level orders the levels.
#include "bgcr_internal.h"

namespace bgcr {

namespace {

__device__ inline double over(double a, double b) { return a / b; }
__device__ inline zd over(zd a, zd b) {
    const double d = b.x * b.x + b.y * b.y;
    return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

constexpr int ILU_NT = 256;

// Numeric ILU(0) of the rows of one level (one thread per row): for each
// k < i in row i's pattern, in increasing order, l_ik = a_ik / u_kk and
// a_ij -= l_ik u_kj for the j > k that rows i and k both hold (merge of the
// two sorted column lists); updates outside the pattern are dropped.  Rows k
// belong to earlier levels and are final.  A zero or non-finite pivot sets
// *err (plain vector store; every writer stores the same value).
template <class T>
__global__ __launch_bounds__(ILU_NT) void k_ilu0_rows(const int* __restrict__ rows, int nrows,
                                                      const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const int* __restrict__ diag, T* lu, int* err) {
    const int t = blockIdx.x * ILU_NT + threadIdx.x;
    if (t >= nrows) return;
    const int i = rows[t];
    const int e1 = rp[i + 1], di = diag[i];
    for (int e = rp[i]; e < di; ++e) {
        const int k = ci[e];
        const int dk = diag[k];
        const T ukk = lu[dk];
        const double mag = absq(ukk);
        if (!(mag > 0.0) || !isfinite(mag)) {
            *err = 1;
            return;
        }
        const T lik = over(lu[e], ukk);
        lu[e] = lik;
        int f = e + 1, g = dk + 1;
        const int gend = rp[k + 1];
        while (f < e1 && g < gend) {
            const int cf = ci[f], cg = ci[g];
            if (cf == cg) {
                lu[f] -= lik * lu[g];
                ++f;
                ++g;
            } else if (cf < cg) {
                ++f;
            } else {
                ++g;
            }
        }
    }
    const double dd = absq(lu[di]);
    if (!(dd > 0.0) || !isfinite(dd)) *err = 1;
}

// One level of a triangular solve with P right-hand sides (row-major blocks,
// leading dimension P): P consecutive threads share a row, one column each.
// LOWER: y_i = in_i - sum_{k < i} l_ik y_k (unit diagonal);
// upper: x_i = (in_i - sum_{j > i} u_ij x_j) / u_ii.  The referenced rows of
// `out` are final (earlier levels).  `in` may alias `out`: each thread reads
// its own entry before it writes it, and no other thread of the level touches
// that entry.
template <class T, int P, bool LOWER>
__global__ __launch_bounds__(ILU_NT) void k_trsv_rows(const int* __restrict__ rows, int nrows,
                                                      const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const int* __restrict__ diag, const T* __restrict__ lu,
                                                      const T* in, T* out, const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    const int t = blockIdx.x * ILU_NT + threadIdx.x;
    const int r = t / P, c = t % P;
    if (r >= nrows) return;
    const int i = rows[r];
    T s = in[(int64_t)i * P + c];
    if constexpr (LOWER) {
        const int e1 = diag[i];
        for (int e = rp[i]; e < e1; ++e) s -= lu[e] * out[(int64_t)ci[e] * P + c];
        out[(int64_t)i * P + c] = s;
    } else {
        const int d = diag[i], e1 = rp[i + 1];
        for (int e = d + 1; e < e1; ++e) s -= lu[e] * out[(int64_t)ci[e] * P + c];
        out[(int64_t)i * P + c] = over(s, lu[d]);
    }
}

// *diff = 1 where two CSR patterns of the same n and nnz differ (the flag is
// cleared by the caller; every writer stores the same value)
__global__ __launch_bounds__(ILU_NT) void k_pattern_diff(int64_t n, int64_t nnz, const int* __restrict__ rpa,
                                                         const int* __restrict__ cia, const int* __restrict__ rpb,
                                                         const int* __restrict__ cib, int* diff) {
    const int64_t stride = (int64_t)gridDim.x * ILU_NT;
    bool d = false;
    for (int64_t e = (int64_t)blockIdx.x * ILU_NT + threadIdx.x; e < nnz; e += stride) d |= cia[e] != cib[e];
    for (int64_t e = (int64_t)blockIdx.x * ILU_NT + threadIdx.x; e <= n; e += stride) d |= rpa[e] != rpb[e];
    if (d) *diff = 1;
}

// out = in M row by row (M: P x P, row-major, FP64 or complex128)
template <class T, int P>
__global__ __launch_bounds__(ILU_NT) void k_rows_times(int64_t n, const T* __restrict__ in,
                                                       const acc_t<T>* __restrict__ M, T* __restrict__ out,
                                                       const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    __shared__ acc_t<T> Ms[P * P];
    for (int e = threadIdx.x; e < P * P; e += ILU_NT) Ms[e] = M[e];
    __syncthreads();
    const int64_t total = n * P, stride = (int64_t)gridDim.x * ILU_NT;
    for (int64_t t = (int64_t)blockIdx.x * ILU_NT + threadIdx.x; t < total; t += stride) {
        const int64_t r = t / P;
        const int c = (int)(t % P);
        acc_t<T> s = zero<acc_t<T>>();
        for (int a = 0; a < P; ++a) s += widen(in[r * P + a]) * Ms[a * P + c];
        out[t] = narrow<T>(s);
    }
}

inline int blocks_for(int64_t work) {
    const int64_t b = (work + ILU_NT - 1) / ILU_NT;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <class T>
hipError_t ilu0_level(hipStream_t st, const int* rows, int nrows, const int* rp, const int* ci, const int* diag,
                      T* lu, int* err) {
    if (nrows <= 0) return hipSuccess;
    k_ilu0_rows<T><<<blocks_for(nrows), ILU_NT, 0, st>>>(rows, nrows, rp, ci, diag, lu, err);
    return hipGetLastError();
}

template <class T>
hipError_t trsv_level(hipStream_t st, int P, bool lower, const int* rows, int nrows, const int* rp, const int* ci,
                      const int* diag, const T* lu, const T* in, T* out, const Ctl* ctl) {
    if (nrows <= 0) return hipSuccess;
    const int g = blocks_for((int64_t)nrows * P);
#define BGCR_TRSV(PP)                                                                                            \
    case PP:                                                                                                     \
        if (lower)                                                                                               \
            k_trsv_rows<T, PP, true><<<g, ILU_NT, 0, st>>>(rows, nrows, rp, ci, diag, lu, in, out, ctl);         \
        else                                                                                                     \
            k_trsv_rows<T, PP, false><<<g, ILU_NT, 0, st>>>(rows, nrows, rp, ci, diag, lu, in, out, ctl);        \
        break;
    switch (P) {
        BGCR_TRSV(1)
        BGCR_TRSV(2)
        BGCR_TRSV(4)
        BGCR_TRSV(8)
        BGCR_TRSV(16)
        default:
            return hipErrorNotSupported;
    }
#undef BGCR_TRSV
    return hipGetLastError();
}

hipError_t pattern_diff(hipStream_t st, int64_t n, int64_t nnz, const int* rpa, const int* cia, const int* rpb,
                        const int* cib, int* diff) {
    const int64_t work = nnz > n + 1 ? nnz : n + 1;
    int g = blocks_for(work);
    if (g > 2048) g = 2048;
    k_pattern_diff<<<g, ILU_NT, 0, st>>>(n, nnz, rpa, cia, rpb, cib, diff);
    return hipGetLastError();
}

template <class T>
hipError_t rows_times(hipStream_t st, int P, int64_t n, const T* in, const acc_t<T>* M, T* out, const Ctl* ctl) {
    int g = blocks_for(n * P);
    if (g > 4096) g = 4096;
    switch (P) {
        case 1: k_rows_times<T, 1><<<g, ILU_NT, 0, st>>>(n, in, M, out, ctl); break;
        case 2: k_rows_times<T, 2><<<g, ILU_NT, 0, st>>>(n, in, M, out, ctl); break;
        case 4: k_rows_times<T, 4><<<g, ILU_NT, 0, st>>>(n, in, M, out, ctl); break;
        case 8: k_rows_times<T, 8><<<g, ILU_NT, 0, st>>>(n, in, M, out, ctl); break;
        case 16: k_rows_times<T, 16><<<g, ILU_NT, 0, st>>>(n, in, M, out, ctl); break;
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template hipError_t ilu0_level<double>(hipStream_t, const int*, int, const int*, const int*, const int*, double*,
                                       int*);
template hipError_t ilu0_level<zd>(hipStream_t, const int*, int, const int*, const int*, const int*, zd*, int*);
template hipError_t trsv_level<double>(hipStream_t, int, bool, const int*, int, const int*, const int*, const int*,
                                       const double*, const double*, double*, const Ctl*);
template hipError_t trsv_level<zd>(hipStream_t, int, bool, const int*, int, const int*, const int*, const int*,
                                   const zd*, const zd*, zd*, const Ctl*);
template hipError_t rows_times<double>(hipStream_t, int, int64_t, const double*, const double*, double*,
                                       const Ctl*);
template hipError_t rows_times<zd>(hipStream_t, int, int64_t, const zd*, const zd*, zd*, const Ctl*);

}  // namespace bgcr
