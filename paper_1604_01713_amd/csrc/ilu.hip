// ILU(0) right preconditioning (the incomplete LU factorization the paper
// applies to every system of its convergence experiments, Sections 6.1 and
// 6.2): the numeric factorization and the two triangular solves of
// M^{-1} = U^{-1} L^{-1}, level-scheduled.
//
// The factors share the CSR pattern of A: `lu` holds the strictly lower part
// of L (unit diagonal implied) and the upper part of U, entry for entry where
// A has its nonzeros, with diag[i] the position of (i, i).  A row's level in
// L is one more than the largest level of the rows its strictly lower part
// refers to (in U the same with the strictly upper part), so the rows of one
// level depend only on earlier levels.  The factorization (once per system)
// takes one launch per level; each triangular solve (several per restart
// cycle) is one launch in which rows wait for the values they need.
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
    if (i < 0) return;  // padding of a level
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

// ---------------------------------------------------------------------------
// Triangular solve in one launch, driven by the data.  Every entry of the
// output block starts as PENDING, a signalling NaN whose payload no
// arithmetic produces (arithmetic returns quiet NaNs), and is written exactly
// once, with a coherent 8-byte store, when its row is solved.  A row reads
// each entry it depends on with coherent loads until it is no longer PENDING;
// the value it waited for is the value it uses, so no flag and no fence is
// needed.  The rows are taken in level order, each level padded to whole
// chunks of ILU_NT / P rows (padding entries are -1), and workgroups take the
// chunks in order by an atomic ticket: every row a chunk depends on lies in
// an earlier level, hence an earlier chunk, held by a workgroup that is
// already running, and no row depends on a row of its own chunk.  The solve
// cannot deadlock whatever order the hardware starts workgroups in.  Every
// wait is bounded in time (WAIT_TICKS of the device wall clock, about 0.1 s
// at its 100 MHz, far beyond any legitimate wait); on expiry, or once any
// other wait of the launch has expired (*err, checked every 64 polls), the
// value is taken as a quiet NaN, so every wave ends quickly.
// The launch also re-arms the other block for the next launch (its entries
// of `rearm` set to PENDING, the other ticket counter to 0).
// ---------------------------------------------------------------------------
constexpr unsigned long long PENDING = 0x7FF4DEADBEEF0001ull;
constexpr unsigned long long QNAN = 0x7FF8000000000000ull;
constexpr unsigned long long WAIT_TICKS = 10000000ull;
constexpr int MAXD = 8;  // dependencies of a row requested together (longer rows poll one at a time)

__device__ inline unsigned long long ld_coherent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_coherent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_flag(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void raise_flag(int* p) { __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// an entry of T as 8-byte words: false while any word is PENDING
__device__ inline bool ready(const double* p, double& v) {
    const unsigned long long w = ld_coherent((const unsigned long long*)p);
    v = __builtin_bit_cast(double, w);
    return w != PENDING;
}
__device__ inline bool ready(const zd* p, zd& v) {
    const unsigned long long a = ld_coherent((const unsigned long long*)p);
    const unsigned long long b = ld_coherent((const unsigned long long*)p + 1);
    v = {__builtin_bit_cast(double, a), __builtin_bit_cast(double, b)};
    return a != PENDING && b != PENDING;
}
__device__ inline void publish(double* p, double v) {
    st_coherent((unsigned long long*)p, __builtin_bit_cast(unsigned long long, v));
}
__device__ inline void publish(zd* p, zd v) {
    st_coherent((unsigned long long*)p, __builtin_bit_cast(unsigned long long, v.x));
    st_coherent((unsigned long long*)p + 1, __builtin_bit_cast(unsigned long long, v.y));
}
__device__ inline void set_pending(double* p) { *(unsigned long long*)p = PENDING; }
__device__ inline void set_pending(zd* p) {
    ((unsigned long long*)p)[0] = PENDING;
    ((unsigned long long*)p)[1] = PENDING;
}
template <class T>
__device__ inline T from_words(const unsigned long long (&w)[sizeof(T) / 8]);
template <>
__device__ inline double from_words<double>(const unsigned long long (&w)[1]) {
    return __builtin_bit_cast(double, w[0]);
}
template <>
__device__ inline zd from_words<zd>(const unsigned long long (&w)[2]) {
    return {__builtin_bit_cast(double, w[0]), __builtin_bit_cast(double, w[1])};
}
__device__ inline void quiet_nan(double& v) { v = __builtin_bit_cast(double, QNAN); }
__device__ inline void quiet_nan(zd& v) { v = {__builtin_bit_cast(double, QNAN), __builtin_bit_cast(double, QNAN)}; }

// one row (and column c) of the data-driven solve; see k_trsv_flow
template <class T, int P, bool LOWER>
__device__ inline void trsv_row(int i, int c, const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ diag, const T* __restrict__ lu, const T* in, T* out,
                                T* rearm, int* err) {
    const int64_t me = (int64_t)i * P + c;
    const T b = in[me];
    const int d = diag[i];
    const int e0 = LOWER ? rp[i] : d + 1;
    const int e1 = LOWER ? d : rp[i + 1];
    T s = b;
    const int nd = e1 - e0;
    if (nd > 0 && nd <= MAXD) {
        // all dependencies requested at once (one round trip when they are
        // ready), then only the missing ones polled again.  The loads are
        // unconditional, slots past nd repeating the last dependency, so
        // that they issue back to back.
        constexpr int W = sizeof(T) / 8;
        const unsigned long long* addr[MAXD];
        unsigned long long wv[MAXD][W];
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
            addr[k] = (const unsigned long long*)(out + (int64_t)ci[e0 + (k < nd ? k : nd - 1)] * P + c);
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
#pragma unroll
            for (int j = 0; j < W; ++j) wv[k][j] = ld_coherent(addr[k] + j);
        unsigned pend = 0;
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
#pragma unroll
            for (int j = 0; j < W; ++j)
                if (k < nd && wv[k][j] == PENDING) pend |= 1u << k;
        if (pend) {
            const unsigned long long t0 = wall_clock64();
            unsigned spins = 0;
            while (pend) {
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int k = 0; k < MAXD; ++k)
                    if ((pend >> k) & 1u) {
                        bool got = true;
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            wv[k][j] = ld_coherent(addr[k] + j);
                            got = got && wv[k][j] != PENDING;
                        }
                        if (got) pend &= ~(1u << k);
                    }
                if (pend && (++spins & 63u) == 0 && (ld_flag(err) != 0 || wall_clock64() - t0 > WAIT_TICKS)) {
#pragma unroll
                    for (int k = 0; k < MAXD; ++k)
                        if ((pend >> k) & 1u)
#pragma unroll
                            for (int j = 0; j < W; ++j) wv[k][j] = QNAN;
                    raise_flag(err);
                    pend = 0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            const T l = lu[e0 + (k < nd ? k : nd - 1)];
            if (k < nd) s -= l * from_words<T>(wv[k]);
        }
    } else if (nd > MAXD) {
        for (int e = e0; e < e1; ++e) {
            const T* q = out + (int64_t)ci[e] * P + c;
            T v;
            if (!ready(q, v)) {
                const unsigned long long t0 = wall_clock64();
                unsigned spins = 0;
                while (!ready(q, v)) {
                    if ((++spins & 63u) == 0 && (ld_flag(err) != 0 || wall_clock64() - t0 > WAIT_TICKS)) {
                        quiet_nan(v);
                        raise_flag(err);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            s -= lu[e] * v;
        }
    }
    publish(out + me, LOWER ? s : over(s, lu[d]));
    // re-arm the other block for the next launch (after `b` has been used:
    // `in` may be that block)
    set_pending(rearm + me);
}

template <class T, int P, bool LOWER>
__global__ __launch_bounds__(ILU_NT) void k_trsv_flow(int64_t npad, const int* __restrict__ ord,
                                                      const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const int* __restrict__ diag, const T* __restrict__ lu,
                                                      const T* in, T* out, T* rearm, unsigned* tick,
                                                      unsigned* tick_next, int* err, const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    __shared__ unsigned chunk;
    if (blockIdx.x == 0 && threadIdx.x == 0) *tick_next = 0u;
    constexpr int R = ILU_NT / P;
    const int64_t nchunks = npad / R;
    const int c = threadIdx.x % P;
    // a fixed grid of workgroups, each taking chunks by ticket until none is
    // left; a workgroup takes its next chunk only when all rows of the
    // current one are written
    for (;;) {
        if (threadIdx.x == 0) chunk = atomicAdd(tick, 1u);
        __syncthreads();
        const int64_t my = chunk;
        __syncthreads();
        if (my >= nchunks) break;
        const int i = ord[my * R + threadIdx.x / P];
        if (i >= 0) trsv_row<T, P, LOWER>(i, c, rp, ci, diag, lu, in, out, rearm, err);  // -1: padding
    }
}

// every entry of an n x P block set to PENDING
template <class T>
__global__ __launch_bounds__(ILU_NT) void k_fill_pending(int64_t count, T* y) {
    const int64_t stride = (int64_t)gridDim.x * ILU_NT;
    for (int64_t t = (int64_t)blockIdx.x * ILU_NT + threadIdx.x; t < count; t += stride) set_pending(y + t);
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
hipError_t trsv_flow(hipStream_t st, int P, bool lower, int64_t npad, const int* ord, const int* rp, const int* ci,
                     const int* diag, const T* lu, const T* in, T* out, T* rearm, unsigned* tick, unsigned* tick_next,
                     int* err, const Ctl* ctl) {
    if (npad <= 0) return hipSuccess;
    // two workgroups per compute unit: a level of the 128^3 stencil holds up
    // to a few hundred chunks; more resident waiters only add polling (512,
    // 1024 and 2048 workgroups measured 2.6, 2.7 and 3.0 ms per M^{-1} at
    // p = 8, whatever the poll interval)
    const int64_t nchunks = npad / (ILU_NT / P);
    const int g = (int)(nchunks < 512 ? nchunks : 512);
#define BGCR_FLOW(PP)                                                                                            \
    case PP:                                                                                                     \
        if (lower)                                                                                               \
            k_trsv_flow<T, PP, true><<<g, ILU_NT, 0, st>>>(npad, ord, rp, ci, diag, lu, in, out, rearm, tick,       \
                                                           tick_next, err, ctl);                                 \
        else                                                                                                     \
            k_trsv_flow<T, PP, false><<<g, ILU_NT, 0, st>>>(npad, ord, rp, ci, diag, lu, in, out, rearm, tick,      \
                                                            tick_next, err, ctl);                                \
        break;
    switch (P) {
        BGCR_FLOW(1)
        BGCR_FLOW(2)
        BGCR_FLOW(4)
        BGCR_FLOW(8)
        BGCR_FLOW(16)
        default:
            return hipErrorNotSupported;
    }
#undef BGCR_FLOW
    return hipGetLastError();
}

template <class T>
hipError_t fill_pending(hipStream_t st, int64_t count, T* y) {
    if (count <= 0) return hipSuccess;
    int g = blocks_for(count);
    if (g > 4096) g = 4096;
    k_fill_pending<T><<<g, ILU_NT, 0, st>>>(count, y);
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
template hipError_t trsv_flow<double>(hipStream_t, int, bool, int64_t, const int*, const int*, const int*, const int*,
                                      const double*, const double*, double*, double*, unsigned*, unsigned*, int*,
                                      const Ctl*);
template hipError_t trsv_flow<zd>(hipStream_t, int, bool, int64_t, const int*, const int*, const int*, const int*,
                                  const zd*, const zd*, zd*, zd*, unsigned*, unsigned*, int*, const Ctl*);
template hipError_t fill_pending<double>(hipStream_t, int64_t, double*);
template hipError_t fill_pending<zd>(hipStream_t, int64_t, zd*);
template hipError_t rows_times<double>(hipStream_t, int, int64_t, const double*, const double*, double*,
                                       const Ctl*);
template hipError_t rows_times<zd>(hipStream_t, int, int64_t, const zd*, const zd*, zd*, const Ctl*);

}  // namespace bgcr
