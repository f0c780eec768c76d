// HIP kernels of the block GCRO-DR restart cycle for gfx950 (MI355X).
//
// Data layout: every n x P block (basis block V_j, SpMM output W, recycled
// column blocks of U and C, residual R) is row-major with leading dimension P,
// so one row of a block is P contiguous scalars and a tile of NT/P rows of a
// block is NT contiguous scalars.  A streaming kernel gives each workgroup a
// contiguous range of row tiles; workgroups are renumbered so that each of the
// 8 XCDs owns one contiguous slice of rows (L2 locality for the SpMM gathers).
//
// Reductions over rows are two-stage and deterministic: a workgroup writes
// its partial sums to part[wg][*]; a second kernel sums them in fixed order.
#include <mutex>
#include <type_traits>

#include "bgcr_internal.h"
#include "spmm_sweep.h"

namespace bgcr {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
template <class A> __host__ __device__ inline A from_real_h(double v);
template <> __host__ __device__ inline double from_real_h<double>(double v) { return v; }
template <> __host__ __device__ inline zd from_real_h<zd>(double v) { return {v, 0.0}; }

template <class T> __host__ __device__ inline T tz();
template <> __host__ __device__ inline float tz<float>() { return 0.f; }
template <> __host__ __device__ inline double tz<double>() { return 0.0; }
template <> __host__ __device__ inline zd tz<zd>() { return {0.0, 0.0}; }
template <> __host__ __device__ inline bf16 tz<bf16>() { return bf16{0}; }

__device__ inline double inv_real(double a) { return 1.0 / a; }
__device__ inline double scale_by(double s, double a) { return s * a; }
__device__ inline zd scale_by(double s, zd a) { return {s * a.x, s * a.y}; }
template <class A> __device__ inline A from_real(double v);
template <> __device__ inline double from_real<double>(double v) { return v; }
template <> __device__ inline zd from_real<zd>(double v) { return {v, 0.0}; }
template <> __device__ inline float from_real<float>(double v) { return (float)v; }

template <class TO, class TI> __host__ __device__ inline TO conv(TI v);
template <> __host__ __device__ inline double conv<double, double>(double v) { return v; }
template <> __host__ __device__ inline float conv<float, double>(double v) { return (float)v; }
template <> __host__ __device__ inline double conv<double, float>(float v) { return (double)v; }
template <> __host__ __device__ inline float conv<float, float>(float v) { return v; }
template <> __host__ __device__ inline zd conv<zd, zd>(zd v) { return v; }
template <> __host__ __device__ inline double conv<double, bf16>(bf16 v) { return widen(v); }
template <> __host__ __device__ inline bf16 conv<bf16, double>(double v) { return narrow<bf16>(v); }

// Workgroup renumbering: hardware dispatches workgroup w to XCD w % 8; the
// logical index gives XCD x the contiguous logical range [x G/8, (x+1) G/8).
__device__ inline int logical_wg() {
    const int w = blockIdx.x, G = gridDim.x;
    if (G % 8 != 0) return w;
    return (w % 8) * (G / 8) + (w / 8);
}

__device__ inline void tile_range(int64_t ntiles, int lw, int64_t& t0, int64_t& t1) {
    const int64_t G = gridDim.x;
    t0 = (int64_t)lw * ntiles / G;
    t1 = (int64_t)(lw + 1) * ntiles / G;
}

// Contribution of one row tile to one output of a tall-skinny product.
// Output o < ndot: (Q column c = o / P)^H (W column o % P) with the Q tile of
// block c / P at Qs[(c/P)*NT ...]; o >= ndot: Gram entry (a, b) of the W tile.
template <class T, int P>
__device__ inline acc_t<T> tile_item(const T* Qs, const T* Ws, int ndot, int o, int g, int G) {
    constexpr int ROWS = NT / P;
    using A = acc_t<T>;
    A s = zero<A>();
    const int bb = o % P;
    const T* x;
    if (o < ndot) {
        const int c = o / P;
        x = Qs + (c / P) * NT + (c % P);
    } else {
        x = Ws + (o - ndot) / P;
    }
    const T* y = Ws + bb;
    for (int rr = g; rr < ROWS; rr += G) s += cj(widen(x[rr * P])) * widen(y[rr * P]);
    return s;
}

// Item bookkeeping shared by the dot kernels: nout outputs, G row groups per
// output when nout < NT, thread t owns items t + NT*i.
struct Items {
    int nout, G, items;
    __device__ Items(int nout_) : nout(nout_) {
        G = (nout > 0 && nout < NT) ? NT / nout : 1;
        items = nout * G;
    }
};

template <class A>
__device__ inline void write_partials(const Items& it, A (&acc)[MAXI], A* red, A* part, int lw) {
    const int t = threadIdx.x;
    if (it.nout == 0) return;
    if (it.G == 1) {
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            const int id = t + NT * i;
            if (id < it.items) part[(int64_t)lw * it.nout + id] = acc[i];
        }
        return;
    }
    __syncthreads();
    if (t < it.items) red[t] = acc[0];
    __syncthreads();
    if (t < it.nout) {
        A s = zero<A>();
        for (int g = 0; g < it.G; ++g) s += red[g * it.nout + t];
        part[(int64_t)lw * it.nout + t] = s;
    }
}

// ---------------------------------------------------------------------------
// sweep 1: block SpMM fused with the first block-CGS dot products
// ---------------------------------------------------------------------------
// W = (A Vin) Rinv and Vout = Vin Rinv for the rows of each tile; the dot
// part accumulates [Q_0 .. Q_{nq-1}, Vout]^H W (Vout from the tile itself).
template <class T, int P>
__device__ __forceinline__ void spmm_dot_body(int64_t n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const T* __restrict__ av, const T* __restrict__ Vin,
                                              const acc_t<T>* __restrict__ Rinv, T* Vout, T* Wout,
                                              const BlockPtrs& Q, int nq, int with_self,
                                              acc_t<T>* __restrict__ part, const Ctl* ctl) {
    using A = acc_t<T>;
    if (ctl && ctl->active == 0) return;
    constexpr int ROWS = NT / P;
    extern __shared__ __align__(16) unsigned char smem[];
    A* raw = (A*)smem;
    A* Rs = raw + NT;
    T* Ws = (T*)(Rs + P * P);
    T* Qs = Ws + NT;
    const int t = threadIdx.x, r = t / P, b = t % P;
    const int nqt = nq + with_self;
    const Items it(nqt * P * P);
    A acc[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) acc[i] = zero<A>();
    if (Rinv && t < P * P) Rs[t] = Rinv[t];
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_range((n + ROWS - 1) / ROWS, lw, t0, t1);
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t row = tile * ROWS + r;
        const bool ok = row < n;
        A s = zero<A>();
        if (ok) {
            const int e = rp[row + 1];
            for (int kk = rp[row]; kk < e; ++kk) s += widen(av[kk]) * widen(Vin[(int64_t)ci[kk] * P + b]);
        }
        A w = s;
        if (Rinv) {
            raw[t] = s;
            __syncthreads();
            w = zero<A>();
#pragma unroll
            for (int a = 0; a < P; ++a) w += raw[r * P + a] * Rs[a * P + b];
        }
        const T wt = narrow<T>(w);
        Ws[t] = wt;
        if (ok) Wout[row * P + b] = wt;
        if (Vout) {
            A v = zero<A>();
            if (ok) {
                if (Rinv) {
#pragma unroll
                    for (int a = 0; a < P; ++a) v += widen(Vin[row * P + a]) * Rs[a * P + b];
                } else {
                    v = widen(Vin[row * P + b]);
                }
            }
            const T vt = narrow<T>(v);
            if (ok) Vout[row * P + b] = vt;
            if (with_self) Qs[nq * NT + t] = vt;
        }
        for (int i = 0; i < nq; ++i) Qs[i * NT + t] = ok ? ((const T*)Q.p[i])[row * P + b] : tz<T>();
        __syncthreads();
        if (it.nout) {
#pragma unroll
            for (int i = 0; i < MAXI; ++i) {
                const int id = t + NT * i;
                if (id < it.items) acc[i] += tile_item<T, P>(Qs, Ws, it.nout, id % it.nout, id / it.nout, it.G);
            }
        }
        __syncthreads();
    }
    write_partials(it, acc, raw, part, lw);
}

// sweep 1 of a block Arnoldi step
template <class T, int P>
__global__ __launch_bounds__(NT) void k_spmm_dot(int64_t n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const T* __restrict__ av, const T* __restrict__ Vin,
                                                 const acc_t<T>* __restrict__ Rinv, T* Vout, T* Wout, BlockPtrs Q,
                                                 int nq, int with_self, acc_t<T>* __restrict__ part, const Ctl* ctl) {
    spmm_dot_body<T, P>(n, rp, ci, av, Vin, Rinv, Vout, Wout, Q, nq, with_self, part, ctl);
}

// plain block SpMM W = A V (recycle import A U, standalone entry point)
template <class T, int P>
__global__ __launch_bounds__(NT) void k_spmm(int64_t n, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const T* __restrict__ av, const T* __restrict__ Vin, T* Wout) {
    BlockPtrs none;
    spmm_dot_body<T, P>(n, rp, ci, av, Vin, nullptr, nullptr, Wout, none, 0, 0, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// sweeps 2 and 3: W' = W - Q S (and/or W' = W Rmul), optional store, partial
// Q^H W' and/or Gram W'^H W'
// ---------------------------------------------------------------------------
template <class T, int P>
__device__ __forceinline__ void update_dot_body(int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                                                const acc_t<T>* __restrict__ S, const acc_t<T>* __restrict__ Rmul,
                                                T* Wout, int dot_q, int gram, acc_t<T>* __restrict__ part,
                                                const Ctl* ctl) {
    using A = acc_t<T>;
    if (ctl && ctl->active == 0) return;
    constexpr int ROWS = NT / P;
    extern __shared__ __align__(16) unsigned char smem[];
    A* raw = (A*)smem;
    A* Rs = raw + NT;
    A* Ss = Rs + P * P;
    T* Ws = (T*)(Ss + (S ? nq * P * P : 0));
    T* Qs = Ws + NT;
    const int t = threadIdx.x, r = t / P, b = t % P;
    const int ndot = dot_q ? nq * P * P : 0;
    const Items it(ndot + (gram ? P * P : 0));
    const bool needQ = nq > 0 && (S != nullptr || dot_q);
    A acc[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) acc[i] = zero<A>();
    if (Rmul && t < P * P) Rs[t] = Rmul[t];
    if (S)
        for (int e = t; e < nq * P * P; e += NT) Ss[e] = S[e];
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_range((n + ROWS - 1) / ROWS, lw, t0, t1);
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t row = tile * ROWS + r;
        const bool ok = row < n;
        A w = ok ? widen(Win[row * P + b]) : zero<A>();
        if (needQ)
            for (int i = 0; i < nq; ++i) Qs[i * NT + t] = ok ? ((const T*)Q.p[i])[row * P + b] : tz<T>();
        __syncthreads();
        if (S) {
            for (int c = 0; c < nq * P; ++c) w -= widen(Qs[(c / P) * NT + r * P + (c % P)]) * Ss[c * P + b];
        }
        if (Rmul) {
            raw[t] = w;
            __syncthreads();
            w = zero<A>();
#pragma unroll
            for (int a = 0; a < P; ++a) w += raw[r * P + a] * Rs[a * P + b];
        }
        const T wt = narrow<T>(w);
        Ws[t] = wt;
        if (ok && Wout) Wout[row * P + b] = wt;
        __syncthreads();
        if (it.nout) {
#pragma unroll
            for (int i = 0; i < MAXI; ++i) {
                const int id = t + NT * i;
                if (id < it.items) acc[i] += tile_item<T, P>(Qs, Ws, ndot, id % it.nout, id / it.nout, it.G);
            }
        }
        __syncthreads();
    }
    write_partials(it, acc, raw, part, lw);
}

#define BGCR_UPDATE_KERNEL(NAME)                                                                                   \
    template <class T, int P>                                                                                      \
    __global__ __launch_bounds__(NT) void NAME(int64_t n, const T* Win, BlockPtrs Q, int nq,                       \
                                               const acc_t<T>* __restrict__ S, const acc_t<T>* __restrict__ Rmul,  \
                                               T* Wout, int dot_q, int gram, acc_t<T>* __restrict__ part,           \
                                               const Ctl* ctl) {                                                    \
        update_dot_body<T, P>(n, Win, Q, nq, S, Rmul, Wout, dot_q, gram, part, ctl);                               \
    }
// sweep 2: second block-CGS pass, partial Q^H (W - Q S1)
BGCR_UPDATE_KERNEL(k_proj_dot)
// sweep 3: W'' = W - Q S stored, partial Gram of W''
BGCR_UPDATE_KERNEL(k_proj_gram)
// tall-skinny products outside the Arnoldi step (Gram/normalise of R, recycle dots)
BGCR_UPDATE_KERNEL(k_tsdot)
#undef BGCR_UPDATE_KERNEL

// ---------------------------------------------------------------------------
// block-CGS sweeps of a one-column block (P = 1, real data): one lane per
// row, the next row's NQ + 1 loads in flight while the current row is
// computed.  w' = w - sum_i q_i s_i in FP64 (S null: no update), then DOT:
// partial q_i^T w' (i < nq); otherwise w' stored (as T) and partial w'^T w'.
// The accumulators stay in registers; at the end they are summed over the
// wave with cross-lane exchanges and over the 4 waves in LDS (fixed order).
// Blocks past nq read block 0 with coefficient 0 and their dots are not
// written; rows past n load row n - 1 and are weighted 0.
// ---------------------------------------------------------------------------
template <class T, int NQ, bool DOT>
__global__ __launch_bounds__(NT) void k_narrow_sweep(int64_t n, const T* Win, BlockPtrs Q, int nq,
                                                     const double* __restrict__ S, T* Wout,
                                                     double* __restrict__ part, const Ctl* ctl) {
    static_assert(NT == 256, "4 waves per workgroup");
    constexpr int NO = DOT ? NQ : 1;
    if (ctl && ctl->active == 0) return;
    __shared__ double Ss[NQ];
    __shared__ double red[4][NO];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int e = t; e < NQ; e += NT) Ss[e] = (S && e < nq) ? S[e] : 0.0;
    const T* qp[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) qp[i] = (const T*)(i < nq ? Q.p[i] : Q.p[0]);
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_range((n + NT - 1) / NT, lw, t0, t1);
    T qn[NQ];
    T wn = T(0);
    auto load = [&](int64_t tile) {
        const int64_t r = tile * NT + t;
        const int64_t row = r < n ? r : n - 1;
        wn = Win[row];
#pragma unroll
        for (int i = 0; i < NQ; ++i) qn[i] = qp[i][row];
    };
    if (t0 < t1) load(t0);
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t row = tile * NT + t;
        T qc[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) qc[i] = qn[i];
        const T wc = wn;
        if (tile + 1 < t1) load(tile + 1);
        double w = (double)wc;
#pragma unroll
        for (int i = 0; i < NQ; ++i) w -= (double)qc[i] * Ss[i];
        const T wt = narrow<T>(w);
        if (!DOT && row < n) Wout[row] = wt;
        const double wv = (double)wt * (row < n ? 1.0 : 0.0);
        if constexpr (DOT) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) acc[i] += (double)qc[i] * wv;
        } else {
            acc[0] += wv * wv;
        }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[o] += __shfl_xor(acc[o], off, 64);
    if (lane == 0)
#pragma unroll
        for (int o = 0; o < NO; ++o) red[wave][o] = acc[o];
    __syncthreads();
    const int nout = DOT ? nq : 1;
    for (int e = t; e < nout; e += NT) part[(int64_t)lw * nout + e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
}

// ---------------------------------------------------------------------------
// out_o (+)= sum_i in_i coef[i][o]  (basis updates: solution, residual, recycle refresh)
// ---------------------------------------------------------------------------
// One lane per row: the lane reads the P entries of its row of every input
// block (a wave reads 64 consecutive rows: contiguous) and keeps the OC*P
// outputs of its row in registers.  The coefficients are the same for every
// row, so their loads are wave-uniform (scalar loads).  Layout of coef:
// [nin][P][nout][P], i.e. for input i and its column a the nout*P
// coefficients are contiguous.  Outputs are done in chunks of OC blocks; the
// first `accumulate` output blocks are accumulated, the others overwritten.
// The rows of IG input blocks are loaded together before their products
// (indices past nin load the last block and are skipped, a wave-uniform
// test), so that IG loads per lane are in flight at once.
template <class TI, class TO, int P, int OC>
__global__ __launch_bounds__(NT) void k_combine(int64_t n, BlockPtrs in, int nin, BlockPtrs out, int nout,
                                                const acc_t<TI>* __restrict__ coef, int accumulate) {
    using A = acc_t<TI>;
    constexpr int IG = P <= 2 ? 8 : (P <= 4 ? 4 : 1);
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x; row < n; row += stride) {
        for (int o0 = 0; o0 < nout; o0 += OC) {
            A acc[OC * P];
#pragma unroll
            for (int e = 0; e < OC * P; ++e) acc[e] = zero<A>();
            for (int i0 = 0; i0 < nin; i0 += IG) {
                A xv[IG][P];
#pragma unroll
                for (int g = 0; g < IG; ++g) {
                    const int i = i0 + g < nin ? i0 + g : nin - 1;
                    const TI* x = (const TI*)in.p[i] + row * P;
#pragma unroll
                    for (int a = 0; a < P; ++a) xv[g][a] = widen(x[a]);
                }
#pragma unroll
                for (int g = 0; g < IG; ++g) {
                    if (i0 + g >= nin) break;
                    const A* cf = coef + (int64_t)(i0 + g) * P * nout * P + (int64_t)o0 * P;
#pragma unroll
                    for (int a = 0; a < P; ++a) {
#pragma unroll
                        for (int oo = 0; oo < OC; ++oo) {
                            if (o0 + oo < nout) {
#pragma unroll
                                for (int b = 0; b < P; ++b)
                                    acc[oo * P + b] += xv[g][a] * cf[(int64_t)a * nout * P + oo * P + b];
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int oo = 0; oo < OC; ++oo) {
                if (o0 + oo < nout) {
                    TO* y = (TO*)out.p[o0 + oo] + row * P;
#pragma unroll
                    for (int b = 0; b < P; ++b) {
                        A v = acc[oo * P + b];
                        if (o0 + oo < accumulate) v += widen(y[b]);
                        y[b] = narrow<TO>(v);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// deterministic second-stage reduction
// ---------------------------------------------------------------------------
// out[o] = add[o] + sum_w part[w][o]: 16 outputs x 16 workgroup-groups per
// block; each thread sums one residue class of w in order, then the 16 class
// sums are added in order (deterministic).
template <class A>
__global__ __launch_bounds__(256) void k_reduce(const A* __restrict__ part, int nwg, int nout,
                                                const A* __restrict__ add, int nadd, A* out, const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    __shared__ A red[256];
    const int t = threadIdx.x;
    const int o = blockIdx.x * 16 + (t % 16);
    const int g = t / 16;
    // eight partial sums per thread, so that eight loads are in flight
    // before the first add waits (the partials come from L2, and one chain of
    // dependent loads would be latency bound)
    A s[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = zero<A>();
    if (o < nout) {
        int w = g;
        for (; w + 16 * 7 < nwg; w += 16 * 8) {
            A v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(w + 16 * u) * nout + o];
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] += v[u];
        }
        for (; w < nwg; w += 16) s[0] += part[(int64_t)w * nout + o];
    }
    red[t] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (t < 16 && o < nout) {
        A s = (add && o < nadd) ? add[o] : zero<A>();
        for (int q = 0; q < 16; ++q) s += red[q * 16 + t];
        out[o] = s;
    }
}

// ---------------------------------------------------------------------------
// small FP64 problems on the device (one workgroup)
// ---------------------------------------------------------------------------
__device__ inline double dabs(double a) { return fabs(a); }
__device__ inline double dabs(zd a) { return sqrt(a.x * a.x + a.y * a.y); }

// Cholesky factor G = R^H R (R upper triangular, positive diagonal) and its
// inverse, by the whole group (P * P <= blockDim.x; thread t < P * P owns
// entry (t / P, t % P)), right-looking: after pivot row i is final, every
// trailing entry subtracts its term of that row, so each entry takes its
// updates in the row order of the dot-product form.  The factorisation fails
// on a pivot not above 1e-24 of the largest diagonal entry of G (columns
// numerically dependent to about 1e-12), or not above `rel` times its own
// diagonal entry (a column numerically in the span of the previous ones;
// scale invariant).  *ok (shared) receives the result; sh (shared) holds two
// doubles.  The inverse is formed row by row from the bottom.
template <class A>
__device__ void chol_inv_group(const A* G, A* R, A* Ri, int P, double rel, int* ok, double* sh) {
    const int t = threadIdx.x, a = t / P, b = t % P;
    const bool own = t < P * P;
    if (t == 0) {
        double maxd = 0.0;
        for (int i = 0; i < P; ++i) maxd = fmax(maxd, re(G[i * P + i]));
        sh[0] = maxd;
        *ok = (maxd > 0.0) && isfinite(maxd);
    }
    A w = own ? G[t] : zero<A>();
    __syncthreads();
    if (!*ok) return;
    const double maxd = sh[0];
    for (int i = 0; i < P; ++i) {
        if (own && a == i && b == i) {
            const double dd = re(w);
            const bool good = (dd > 1e-24 * maxd) && (dd > rel * re(G[t])) && isfinite(dd);
            *ok = good;
            sh[1] = good ? sqrt(dd) : 1.0;
        }
        __syncthreads();
        if (!*ok) return;
        if (own && a == i) {
            const double rii = sh[1];
            R[t] = b < i ? zero<A>() : (b == i ? from_real<A>(rii) : scale_by(1.0 / rii, w));
        }
        __syncthreads();
        if (own && a > i && b > i) w -= cj(R[i * P + a]) * R[i * P + b];
    }
    // the inverse, row by row from the bottom
    if (own) Ri[t] = a > b ? zero<A>() : (a == b ? from_real<A>(1.0 / re(R[t])) : zero<A>());
    __syncthreads();
    for (int i = P - 2; i >= 0; --i) {
        if (own && a == i && b > i) {
            A s = zero<A>();
            for (int l = i + 1; l <= b; ++l) s += R[i * P + l] * Ri[l * P + b];
            Ri[t] = scale_by(-1.0 / re(R[i * P + i]), s);
        }
        __syncthreads();
    }
}

template <class A>
__device__ void reduce_small(const A* part, int nwg, int nout, int off, A* out, int cnt) {
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        A s = zero<A>();
        for (int w = 0; w < nwg; ++w) s += part[(int64_t)w * nout + off + e];
        out[e] = s;
    }
}

// first pass of CholQR of the cycle's starting block: Z1 = chol(Gram).
// With an enlarged block (nrhs < P) the block is [r, Z] and its enlarging
// columns are scaled by s with s^2 = |r|^2 / mean |z_j|^2 (the span, hence
// the iterate, is unchanged, while the Gram matrix stays well conditioned
// when |r| has become small): the Gram of [r, s Z] is D G D with
// D = diag(1.., s..), and the update matrix returned is D Z1^{-1}, so that
// [r, Z] (D Z1^{-1}) = [r, s Z] Z1^{-1}.
template <class A, int P>
__global__ void k_cholqr_first(const A* gram, A* Z1, A* Z1inv, int nrhs, Ctl* ctl) {
    __shared__ A Gs[P * P], Rs[P * P], Ri[P * P];
    __shared__ int okf;
    __shared__ double dsc[P], shv[2];
    if (threadIdx.x == 0) {
        double s = 1.0;
        if (nrhs < P) {
            double r2 = 0.0, z2 = 0.0;
            for (int i = 0; i < nrhs; ++i) r2 += re(gram[i * P + i]);
            for (int i = nrhs; i < P; ++i) z2 += re(gram[i * P + i]);
            r2 /= nrhs;
            z2 /= (P - nrhs);
            if (r2 > 0.0 && z2 > 0.0) s = sqrt(r2 / z2);
        }
        for (int i = 0; i < P; ++i) dsc[i] = i < nrhs ? 1.0 : s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P * P; e += blockDim.x) Gs[e] = scale_by(dsc[e / P] * dsc[e % P], gram[e]);
    __syncthreads();
    chol_inv_group(Gs, Rs, Ri, P, 1e-14, &okf, shv);  // CholQR2 needs cond(start block) below about 1e7
    __syncthreads();
    if (!okf) {
        if (threadIdx.x == 0) {
            ctl->active = 0;
            ctl->meff = 0;
            ctl->status = 1;
        }
        return;
    }
    for (int e = threadIdx.x; e < P * P; e += blockDim.x) {
        Z1[e] = Rs[e];
        Z1inv[e] = scale_by(dsc[e / P], Ri[e]);
    }
    if (threadIdx.x == 0) ctl->status = 0;
}

// second pass: Z2 = chol(Gram of R Z1^{-1}); Z = Z2 Z1; LSQ right-hand side
// E Z (Algorithm 1) and the cycle control block are initialised here.
template <class A, int P>
__global__ void k_cholqr_second(const A* gram, const A* Z1, A* Rinv0, A* g, int m, int nrhs, Ctl* ctl) {
    __shared__ A Gs[P * P], Rs[P * P], Ri[P * P];
    __shared__ int okf;
    __shared__ double shv[2];
    if (ctl->status != 0) return;
    for (int e = threadIdx.x; e < P * P; e += blockDim.x) Gs[e] = gram[e];
    __syncthreads();
    chol_inv_group(Gs, Rs, Ri, P, 0.0, &okf, shv);
    __syncthreads();
    if (!okf) {
        if (threadIdx.x == 0) {
            ctl->active = 0;
            ctl->meff = 0;
            ctl->status = 1;
        }
        return;
    }
    for (int e = threadIdx.x; e < P * P; e += blockDim.x) Rinv0[e] = Ri[e];
    for (int e = threadIdx.x; e < (m + 1) * P * P; e += blockDim.x) {
        const int i = e / P, j = e % P;
        // E Z, or with an enlarged block its first column only (E_1 F_0 e_1)
        A z = zero<A>();
        if (i < P && j < nrhs)
            for (int l = 0; l < P; ++l) z += Rs[i * P + l] * Z1[l * P + j];
        g[e] = z;
    }
    if (threadIdx.x == 0) {
        ctl->active = 1;
        ctl->meff = 0;
        ctl->status = 0;
    }
}

// Sum over each aligned group of W lanes (W a power of two up to 32), the same
// value on every lane of the group: rotations and mirrors within 16-lane rows
// and quad permutations (DPP moves, a few cycles each) pair the lanes
// symmetrically, and one cross-lane exchange joins two rows for W = 32.
template <int CTRL>
__device__ inline double dpp_mov(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int W>
__device__ inline double group_sum(double x) {
    static_assert(W >= 1 && W <= 32 && (W & (W - 1)) == 0, "groups of 1 .. 32 lanes");
    if constexpr (W >= 32) x += __shfl_xor(x, 16);
    if constexpr (W >= 16) x += dpp_mov<0x128>(x);  // row_ror:8
    if constexpr (W >= 8) x += dpp_mov<0x141>(x);   // row_half_mirror
    if constexpr (W >= 2) x += dpp_mov<0xB1>(x);    // quad_perm 1,0,3,2
    if constexpr (W >= 4) x += dpp_mov<0x4E>(x);    // quad_perm 2,3,0,1
    return x;
}
template <int W>
__device__ inline zd group_sum(zd x) {
    return zd{group_sum<W>(x.x), group_sum<W>(x.y)};
}

// Per block step j (1-based): CholQR factor of W'' from its Gram partials,
// new column block of the block Hessenberg H (and of F = C^H A W), and the
// progressive block-Householder triangularisation of H with the right-hand
// side update (Section 4.1, Householder reflection storage): the reflectors
// of block column j are accumulated into one 2P x 2P unitary QH_j that later
// columns apply as a single matrix product.
template <class A, int P>
__global__ __launch_bounds__(NT) void k_step_small(const A* gram, const A* S, const A* S1, int KP, int j, int m,
                                                   A* H, A* F, A* Rh, A* QH, A* g, A* RinvAll, double* rho,
                                                   Ctl* ctl, double thresh) {
    if (ctl->active == 0) return;
    constexpr int P2 = 2 * P, SROWS = 32;
    static_assert(P * P <= NT, "one Gram entry per thread");
    __shared__ A Gs[P * P], Rs[P * P], Ri[P * P];
    __shared__ A X[P2 * P], M[P2 * P2], tmp[P2 * P], V[P2];
    __shared__ A Sd[SROWS * P];
    A* const Qs = M;  // reflector of an earlier column; M is set up after the last use
    __shared__ double vv, red[NT], shv[2];
    __shared__ int okf;
    const int t = threadIdx.x;
    const int jc = j - 1;
    const int ldH = m * P;
    if (S1) {
        // Gram of W'' = W' - Q S2 from the second pass's data (Pythagoras,
        // Q^H W'' = 0): W''^H W'' = W'^H W' - S2^H S2 with S2 = S - S1; the
        // rows of S2 are staged in LDS, SROWS at a time, by the whole group
        const int q = KP + j * P;
        A acc = t < P * P ? gram[t] : zero<A>();
        for (int c0 = 0; c0 < q; c0 += SROWS) {
            const int cn = q - c0 < SROWS ? q - c0 : SROWS;
            __syncthreads();
            for (int e = t; e < cn * P; e += NT) Sd[e] = S[c0 * P + e] - S1[c0 * P + e];
            __syncthreads();
            if (t < P * P) {
                const int a = t / P, b = t % P;
                for (int c = 0; c < cn; ++c) acc -= cj(Sd[c * P + a]) * Sd[c * P + b];
            }
        }
        if (t < P * P) Gs[t] = acc;
    } else {
        for (int e = t; e < P * P; e += NT) Gs[e] = gram[e];
    }
    __syncthreads();
    chol_inv_group(Gs, Rs, Ri, P, 0.0, &okf, shv);
    __syncthreads();
    if (!okf) {
        if (t == 0) {
            ctl->active = 0;
            ctl->meff = j - 1;
            ctl->status = 1;
        }
        return;
    }
    for (int e = t; e < P * P; e += NT) RinvAll[(int64_t)j * P * P + e] = Ri[e];
    // new block column of H: rows < jP are the dots against V_1..V_j, rows
    // jP .. (j+1)P - 1 the factor R_j
    auto hcol = [&](int i, int bb) { return (i < j * P) ? S[(KP + i) * P + bb] : Rs[(i - j * P) * P + bb]; };
    for (int e = t; e < (j + 1) * P * P; e += NT) {
        const int i = e / P, bb = e % P;
        H[(int64_t)i * ldH + jc * P + bb] = hcol(i, bb);
    }
    for (int e = t; e < KP * P; e += NT) {
        const int i = e / P, bb = e % P;
        F[(int64_t)i * ldH + jc * P + bb] = S[i * P + bb];
    }
    // apply the stored block reflectors of earlier block columns: reflector i
    // acts on row blocks i-1 and i, so a 2P-row window X slides down the
    // column (its lower block enters unreflected) and the finished upper block
    // of each window is written to Rh
    for (int e = t; e < P2 * P; e += NT) X[e] = hcol(e / P, e % P);
    // the reflector products of earlier columns come from memory one after the
    // other: the next one is loaded into registers while the current one is
    // applied
    constexpr int QPT = (P2 * P2 + NT - 1) / NT;
    A qn[QPT];
    auto qload = [&](int i) {
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int e = t + u * NT;
            qn[u] = e < P2 * P2 ? QH[(int64_t)(i - 1) * P2 * P2 + e] : zero<A>();
        }
    };
    if (j > 1) qload(1);
    for (int i = 1; i < j; ++i) {
#pragma unroll
        for (int u = 0; u < QPT; ++u)
            if (t + u * NT < P2 * P2) Qs[t + u * NT] = qn[u];
        __syncthreads();
        if (i + 1 < j) qload(i + 1);
        for (int e = t; e < P2 * P; e += NT) {
            const int rr = e / P, bb = e % P;
            A s = zero<A>();
            for (int l = 0; l < P2; ++l) s += Qs[rr * P2 + l] * X[l * P + bb];
            tmp[e] = s;
        }
        __syncthreads();
        const int r0 = (i - 1) * P;
        for (int e = t; e < P * P; e += NT) {
            Rh[(int64_t)(r0 + e / P) * ldH + jc * P + e % P] = tmp[e];
            X[e] = tmp[P * P + e];
            X[P * P + e] = hcol((i + 1) * P + e / P, e % P);
        }
    }
    __syncthreads();
    // Householder QR of the 2P x P block in rows (j-1)P .. (j+1)P-1 (now in X)
    const int r0 = (j - 1) * P;
    for (int e = t; e < P2 * P2; e += NT) M[e] = from_real<A>((e / P2) == (e % P2) ? 1.0 : 0.0);
    __syncthreads();
    static_assert(P2 <= 64, "one lane of the first wave per row of the 2P x P block");
    for (int c = 0; c < P; ++c) {
        // reflector of column c by the first wave, one lane per row: norms by
        // group sums over the 2P lanes of the rows (every lane of the group
        // ends with the same sum)
        if (t < 64) {
            const int l = t;
            const A xl = (l >= c && l < P2) ? X[l * P + c] : zero<A>();
            const double a2 = group_sum<P2>(absq(xl));
            const double al = sqrt(a2);
            double s2 = 0.0;
            if (al > 0.0) {
                const A x0 = X[c * P + c];
                const double ax = dabs(x0);
                const A ph = ax > 0.0 ? scale_by(1.0 / ax, x0) : from_real<A>(1.0);
                const A beta = scale_by(-al, ph);
                const A vl = l < c ? zero<A>() : (l == c ? x0 - beta : xl);
                if (l < P2) V[l] = vl;
                s2 = group_sum<P2>(absq(vl));
            }
            if (l == 0) vv = s2;
        }
        __syncthreads();
        if (vv > 0.0) {
            // apply the reflector to the window (its columns c..P-1) and to M:
            // one entry per thread, the rows of a column on 2P consecutive
            // lanes, whose v^H x is their group sum (rows above c have v = 0)
            const double f = 2.0 / vv;
            for (int e = t; e < P * P2; e += NT) {
                const int col = e / P2, r = e % P2;
                const A x = X[r * P + col];
                const A w = group_sum<P2>(cj(V[r]) * x);
                if (col >= c) X[r * P + col] = x - scale_by(f, V[r] * w);
            }
            for (int e = t; e < P2 * P2; e += NT) {
                const int col = e / P2, r = e % P2;
                const A x = M[r * P2 + col];
                const A w = group_sum<P2>(cj(V[r]) * x);
                M[r * P2 + col] = x - scale_by(f, V[r] * w);
            }
        }
        __syncthreads();
    }
    for (int e = t; e < P2 * P; e += NT) {
        const int rr = e / P, bb = e % P;
        Rh[(int64_t)(r0 + rr) * ldH + jc * P + bb] = (rr < P && bb >= rr) ? X[e] : zero<A>();
    }
    for (int e = t; e < P2 * P2; e += NT) QH[(int64_t)jc * P2 * P2 + e] = M[e];
    for (int e = t; e < P2 * P; e += NT) tmp[e] = g[(int64_t)(r0 + e / P) * P + e % P];
    __syncthreads();
    for (int e = t; e < P2 * P; e += NT) {
        const int rr = e / P, bb = e % P;
        A s = zero<A>();
        for (int l = 0; l < P2; ++l) s += M[rr * P2 + l] * tmp[l * P + bb];
        g[(int64_t)(r0 + rr) * P + bb] = s;
    }
    __threadfence_block();
    __syncthreads();
    double v = 0.0;
    if (t < P * P) v = absq(g[(int64_t)(j * P + t / P) * P + t % P]);
    red[t] = v;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int q = 0; q < P * P && q < NT; ++q) s += red[q];
        const double rh = sqrt(s);
        rho[jc] = rh;
        ctl->meff = j;
        if (rh <= thresh || j == m) ctl->active = 0;
    }
}

// Enlarging vectors of a single right-hand side (p = 1, block size P):
// columns c0 .. P-1 of the row-major n x P block Y get 2 u - 1, u the top 53
// bits of SplitMix64 (Steele, Lea and Flood 2014; Vigna's finaliser) of the
// counter i + 2^40 c + 2^56 seed, scaled to [0, 1).
__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <class T>
__global__ void k_fill_enlarging(T* __restrict__ Y, int64_t n, int P, int c0, uint64_t seed) {
    const int w = P - c0;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * w) return;
    const int64_t i = e / w;
    const int c = c0 + (int)(e % w);
    const uint64_t ctr = (uint64_t)i + ((uint64_t)c << 40) + (seed << 56);
    const double u = (double)(splitmix64(ctr) >> 11) * (1.0 / 9007199254740992.0);
    Y[i * P + c] = from_real<T>(2.0 * u - 1.0);
}

// S[r][c] = 0 for columns c < ncols of a row-major rows x P matrix
template <class A>
__global__ void k_zero_cols(A* S, int rows, int P, int ncols) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < rows * ncols) S[(e / ncols) * P + e % ncols] = zero<A>();
}

template <class TI, class TO>
__global__ void k_copy_block(int64_t n, int p, const TI* __restrict__ in, int64_t ldi, TO* __restrict__ out,
                             int64_t ldo, int padto) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * padto) return;
    const int64_t i = e / padto;
    const int j = (int)(e % padto);
    out[i * ldo + j] = j < p ? conv<TO, TI>(in[i * ldi + j]) : conv<TO, TI>(tz<TI>());
}

__global__ void k_cast(const double* __restrict__ in, float* __restrict__ out, int64_t nnz) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) out[e] = (float)in[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class F>
static void allow_big_lds(F* f) {
    // gfx950 has 160 KB of LDS per CU; allow a workgroup to use it
    (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

#define BGCR_DISPATCH_P(P, MACRO) \
    switch (P) {                  \
        case 1: MACRO(1); break;  \
        case 2: MACRO(2); break;  \
        case 4: MACRO(4); break;  \
        case 8: MACRO(8); break;  \
        case 16: MACRO(16); break; \
        default: return hipErrorInvalidValue; \
    }

template <class T>
hipError_t Launch<T>::spmm_dot(hipStream_t st, int P, int64_t n, const int* rp, const int* ci, const T* av,
                               const T* Vin, const A* Rinv, T* Vout, T* Wout, const BlockPtrs& Q, int nq,
                               int with_self, A* part, int nwg, const Ctl* ctl) {
    const size_t lds = (size_t)NT * sizeof(A) + (size_t)P * P * sizeof(A) + (size_t)NT * sizeof(T) +
                       (size_t)(nq + with_self) * NT * sizeof(T);
    if ((nq + with_self) * P * P > MAXI * NT) return hipErrorInvalidValue;
    const bool plain = !Rinv && !Vout && nq == 0 && !with_self;
#define L(PP)                                                                                           \
    {                                                                                                   \
        static std::once_flag fl;                                                                       \
        std::call_once(fl, [] { allow_big_lds(k_spmm_dot<T, PP>); allow_big_lds(k_spmm<T, PP>); });     \
        if (plain)                                                                                      \
            hipLaunchKernelGGL((k_spmm<T, PP>), dim3(nwg), dim3(NT), lds, st, n, rp, ci, av, Vin, Wout); \
        else                                                                                            \
            hipLaunchKernelGGL((k_spmm_dot<T, PP>), dim3(nwg), dim3(NT), lds, st, n, rp, ci, av, Vin,    \
                               Rinv, Vout, Wout, Q, nq, with_self, part, ctl);                          \
    }
    BGCR_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <class T>
hipError_t Launch<T>::spmm_rinv(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci,
                                const T* av, const T* Vin, const A* Rinv, T* Vout, T* Wout, const Ctl* ctl) {
    return spmm_block<T, T, T, T>(st, P, n, nnz, rp, ci, av, Vin, Rinv, Vout, Wout, ctl);
}

template <class T>
hipError_t Launch<T>::update_dot(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                                 const A* S, const A* Rmul, T* Wout, int dot_q, int gram, A* part, int nwg,
                                 const Ctl* ctl, int kind) {
    const size_t lds = (size_t)NT * sizeof(A) + (size_t)P * P * sizeof(A) +
                       (S ? (size_t)nq * P * P * sizeof(A) : 0) + (size_t)NT * sizeof(T) +
                       (size_t)nq * NT * sizeof(T);
    if ((dot_q ? nq * P * P : 0) + (gram ? P * P : 0) > MAXI * NT) return hipErrorInvalidValue;
#define L(PP)                                                                                                 \
    {                                                                                                         \
        static std::once_flag fl;                                                                             \
        std::call_once(fl, [] {                                                                               \
            allow_big_lds(k_proj_dot<T, PP>);                                                                 \
            allow_big_lds(k_proj_gram<T, PP>);                                                                \
            allow_big_lds(k_tsdot<T, PP>);                                                                    \
        });                                                                                                   \
        if (kind == 1)                                                                                        \
            hipLaunchKernelGGL((k_proj_dot<T, PP>), dim3(nwg), dim3(NT), lds, st, n, Win, Q, nq, S, Rmul,     \
                               Wout, dot_q, gram, part, ctl);                                                 \
        else if (kind == 2)                                                                                   \
            hipLaunchKernelGGL((k_proj_gram<T, PP>), dim3(nwg), dim3(NT), lds, st, n, Win, Q, nq, S, Rmul,    \
                               Wout, dot_q, gram, part, ctl);                                                 \
        else                                                                                                  \
            hipLaunchKernelGGL((k_tsdot<T, PP>), dim3(nwg), dim3(NT), lds, st, n, Win, Q, nq, S, Rmul, Wout,  \
                               dot_q, gram, part, ctl);                                                       \
    }
    BGCR_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <class T>
template <class TO>
hipError_t Launch<T>::combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out,
                              int nout, const A* coef, int accumulate) {
    const int64_t blocks = (n + NT - 1) / NT;
    const int nwg = (int)(blocks < 2048 ? blocks : 2048);
    // output blocks per pass: 32 accumulators per lane (16 for complex)
    constexpr int ACC = sizeof(A) == 16 ? 16 : 32;
#define OCP(PP) (ACC / PP > 0 ? ACC / PP : 1)
#define L(PP) hipLaunchKernelGGL((k_combine<T, TO, PP, OCP(PP)>), dim3(nwg), dim3(NT), 0, st, n, in, nin, out, nout, coef, accumulate);
    BGCR_DISPATCH_P(P, L)
#undef L
#undef OCP
    return hipGetLastError();
}

template <class A>
hipError_t reduce_partials(hipStream_t st, const A* part, int nwg, int nout, const A* add, A* out, const Ctl* ctl,
                           int nadd) {
    if (nout <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_reduce<A>), dim3((nout + 15) / 16), dim3(256), 0, st, part, nwg, nout, add,
                       nadd < 0 ? nout : nadd, out, ctl);
    return hipGetLastError();
}

template <class TA, class TR>
hipError_t residual(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const TA* av,
                    const TA* B, int64_t ldb, const TA* X, TR* Rout, double* part, int nwg) {
    return residual_rows<TA, TR>(st, P, n, nnz, rp, ci, av, B, ldb, X, Rout, part, nwg);
}

template <class A>
hipError_t cholqr_first(hipStream_t st, int P, const A* gram, A* Z1, A* Z1inv, int nrhs, Ctl* ctl) {
#define L(PP) hipLaunchKernelGGL((k_cholqr_first<A, PP>), dim3(1), dim3(NT), 0, st, gram, Z1, Z1inv, nrhs, ctl);
    BGCR_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <class A>
hipError_t cholqr_second(hipStream_t st, int P, const A* gram, const A* Z1, A* Rinv0, A* g, int m, int nrhs, Ctl* ctl) {
#define L(PP) hipLaunchKernelGGL((k_cholqr_second<A, PP>), dim3(1), dim3(NT), 0, st, gram, Z1, Rinv0, g, m, nrhs, ctl);
    BGCR_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <class A>
hipError_t step_small(hipStream_t st, int P, const A* gram, const A* S, const A* S1, int KP, int j, int m, A* H, A* F,
                      A* Rh, A* QH, A* g, A* RinvAll, double* rho, Ctl* ctl, double thresh) {
#define L(PP) hipLaunchKernelGGL((k_step_small<A, PP>), dim3(1), dim3(NT), 0, st, gram, S, S1, KP, j, m, H, F, Rh, QH, g, RinvAll, rho, ctl, thresh);
    BGCR_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

hipError_t cast_values(hipStream_t st, const double* in, float* out, int64_t nnz) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, in, out, nnz);
    return hipGetLastError();
}

template <class A>
hipError_t zero_cols(hipStream_t st, A* S, int rows, int P, int ncols) {
    if (rows * ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_zero_cols<A>), dim3((rows * ncols + 255) / 256), dim3(256), 0, st, S, rows, P, ncols);
    return hipGetLastError();
}

template <class T>
hipError_t fill_enlarging(hipStream_t st, T* Y, int64_t n, int P, int c0, uint64_t seed) {
    const int64_t tot = n * (P - c0);
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_enlarging<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, n, P, c0, seed);
    return hipGetLastError();
}

template <class TI, class TO>
hipError_t copy_block(hipStream_t st, int64_t n, int p, const TI* in, int64_t ldi, TO* out, int64_t ldo, int padto) {
    const int64_t tot = n * padto;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy_block<TI, TO>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, p, in, ldi,
                       out, ldo, padto);
    return hipGetLastError();
}

template <class T>
hipError_t narrow_sweep(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S, T* Wout,
                        double* part, int nwg, const Ctl* ctl, bool dot) {
    if (nq < 1 || nq > 32 || n < 1 || (!dot && !Wout)) return hipErrorNotSupported;
    const int nb = nq <= 8 ? 8 : (nq <= 16 ? 16 : (nq <= 24 ? 24 : 32));
#define L(NB)                                                                                                      \
    if (dot)                                                                                                       \
        hipLaunchKernelGGL((k_narrow_sweep<T, NB, true>), dim3(nwg), dim3(NT), 0, st, n, Win, Q, nq, S, Wout, part, ctl); \
    else                                                                                                           \
        hipLaunchKernelGGL((k_narrow_sweep<T, NB, false>), dim3(nwg), dim3(NT), 0, st, n, Win, Q, nq, S, Wout, part, ctl)
    switch (nb) {
        case 8: L(8); break;
        case 16: L(16); break;
        case 24: L(24); break;
        default: L(32); break;
    }
#undef L
    return hipGetLastError();
}

// explicit instantiations
template hipError_t narrow_sweep<double>(hipStream_t, int64_t, const double*, const BlockPtrs&, int, const double*,
                                         double*, double*, int, const Ctl*, bool);
template hipError_t narrow_sweep<float>(hipStream_t, int64_t, const float*, const BlockPtrs&, int, const double*,
                                        float*, double*, int, const Ctl*, bool);
template struct Launch<double>;
template struct Launch<float>;
template struct Launch<zd>;
template hipError_t Launch<double>::combine<double>(hipStream_t, int, int64_t, const BlockPtrs&, int,
                                                    const BlockPtrs&, int, const double*, int);
template hipError_t Launch<float>::combine<float>(hipStream_t, int, int64_t, const BlockPtrs&, int,
                                                  const BlockPtrs&, int, const double*, int);
template hipError_t Launch<float>::combine<double>(hipStream_t, int, int64_t, const BlockPtrs&, int,
                                                   const BlockPtrs&, int, const double*, int);
template hipError_t Launch<zd>::combine<zd>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int,
                                            const zd*, int);
template hipError_t reduce_partials<double>(hipStream_t, const double*, int, int, const double*, double*, const Ctl*,
                                            int);
template hipError_t reduce_partials<zd>(hipStream_t, const zd*, int, int, const zd*, zd*, const Ctl*, int);
template hipError_t residual<double, double>(hipStream_t, int, int64_t, int64_t, const int*, const int*, const double*,
                                             const double*, int64_t, const double*, double*, double*, int);
template hipError_t residual<double, float>(hipStream_t, int, int64_t, int64_t, const int*, const int*, const double*,
                                            const double*, int64_t, const double*, float*, double*, int);
template hipError_t residual<zd, zd>(hipStream_t, int, int64_t, int64_t, const int*, const int*, const zd*, const zd*, int64_t,
                                     const zd*, zd*, double*, int);
template hipError_t cholqr_first<double>(hipStream_t, int, const double*, double*, double*, int, Ctl*);
template hipError_t cholqr_first<zd>(hipStream_t, int, const zd*, zd*, zd*, int, Ctl*);
template hipError_t cholqr_second<double>(hipStream_t, int, const double*, const double*, double*, double*, int, int,
                                          Ctl*);
template hipError_t cholqr_second<zd>(hipStream_t, int, const zd*, const zd*, zd*, zd*, int, int, Ctl*);
template hipError_t step_small<double>(hipStream_t, int, const double*, const double*, const double*, int, int, int,
                                       double*, double*, double*, double*, double*, double*, double*, Ctl*, double);
template hipError_t step_small<zd>(hipStream_t, int, const zd*, const zd*, const zd*, int, int, int, zd*, zd*, zd*,
                                   zd*, zd*, zd*, double*, Ctl*, double);
template hipError_t copy_block<double, double>(hipStream_t, int64_t, int, const double*, int64_t, double*, int64_t,
                                               int);
template hipError_t copy_block<zd, zd>(hipStream_t, int64_t, int, const zd*, int64_t, zd*, int64_t, int);
template hipError_t copy_block<float, double>(hipStream_t, int64_t, int, const float*, int64_t, double*, int64_t, int);
template hipError_t copy_block<double, float>(hipStream_t, int64_t, int, const double*, int64_t, float*, int64_t, int);
template hipError_t zero_cols<double>(hipStream_t, double*, int, int, int);
template hipError_t zero_cols<zd>(hipStream_t, zd*, int, int, int);
template hipError_t fill_enlarging<double>(hipStream_t, double*, int64_t, int, int, uint64_t);
template hipError_t fill_enlarging<float>(hipStream_t, float*, int64_t, int, int, uint64_t);
template hipError_t fill_enlarging<zd>(hipStream_t, zd*, int64_t, int, int, uint64_t);
template hipError_t copy_block<bf16, double>(hipStream_t, int64_t, int, const bf16*, int64_t, double*, int64_t, int);
template hipError_t copy_block<double, bf16>(hipStream_t, int64_t, int, const double*, int64_t, bf16*, int64_t, int);

}  // namespace bgcr
