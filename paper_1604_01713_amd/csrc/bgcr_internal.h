// Internal declarations shared by the HIP kernels and the host driver of
// libbgcr.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <complex>

namespace bgcr {

// Interleaved complex double, layout-compatible with std::complex<double>.
struct zd {
    double x, y;
};

__host__ __device__ inline zd operator+(zd a, zd b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline zd operator-(zd a, zd b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline zd operator-(zd a) { return {-a.x, -a.y}; }
__host__ __device__ inline zd operator*(zd a, zd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline zd operator*(double s, zd a) { return {s * a.x, s * a.y}; }
__host__ __device__ inline zd& operator+=(zd& a, zd b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline zd& operator-=(zd& a, zd b) { a.x -= b.x; a.y -= b.y; return a; }

__host__ __device__ inline double cj(double a) { return a; }
__host__ __device__ inline float cj(float a) { return a; }
__host__ __device__ inline zd cj(zd a) { return {a.x, -a.y}; }
__host__ __device__ inline double absq(double a) { return a * a; }
__host__ __device__ inline double absq(zd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double re(double a) { return a; }
__host__ __device__ inline double re(zd a) { return a.x; }

// accumulation / coefficient type of a storage type: FP64 for real storage
// (FP32 basis included), complex128 for complex storage
template <class T> struct acc_of { using type = double; };
template <> struct acc_of<zd> { using type = zd; };
template <class T> using acc_t = typename acc_of<T>::type;

template <class A> __host__ __device__ inline A zero();
template <> __host__ __device__ inline double zero<double>() { return 0.0; }
template <> __host__ __device__ inline zd zero<zd>() { return {0.0, 0.0}; }

__host__ __device__ inline double widen(float v) { return (double)v; }
__host__ __device__ inline double widen(double v) { return v; }
__host__ __device__ inline zd widen(zd v) { return v; }

template <class T> __host__ __device__ inline T narrow(acc_t<T> v);
template <> __host__ __device__ inline float narrow<float>(double v) { return (float)v; }
template <> __host__ __device__ inline double narrow<double>(double v) { return v; }
template <> __host__ __device__ inline zd narrow<zd>(zd v) { return v; }

// BF16 storage scalar: the upper 16 bits of an IEEE binary32.  Used only to
// store basis blocks; every load widens it to FP32 (exact) before arithmetic.
struct bf16 {
    unsigned short u;
};
__host__ __device__ inline float bf16_to_float(bf16 h) { return __builtin_bit_cast(float, (unsigned)h.u << 16); }
// round to nearest, ties to even; NaN stays a (quiet) NaN
__host__ __device__ inline bf16 float_to_bf16(float f) {
    unsigned b = __builtin_bit_cast(unsigned, f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return bf16{(unsigned short)((b >> 16) | 0x40u)};
    b += 0x7fffu + ((b >> 16) & 1u);
    return bf16{(unsigned short)(b >> 16)};
}
__host__ __device__ inline double widen(bf16 v) { return (double)bf16_to_float(v); }
// FP64 -> BF16 rounds through FP32 (the values come from FP32 arithmetic)
template <> __host__ __device__ inline bf16 narrow<bf16>(double v) { return float_to_bf16((float)v); }

// value of a stored scalar in the arithmetic type T (FP32 or FP64)
template <class T> __host__ __device__ inline T as(float v) { return (T)v; }
template <class T> __host__ __device__ inline T as(double v) { return (T)v; }
template <class T> __host__ __device__ inline T as(bf16 v) { return (T)bf16_to_float(v); }
// an FP32/FP64 value in the storage type TO
template <class TO> struct store_of {
    template <class V> __host__ __device__ static TO get(V v) { return (TO)v; }
};
template <> struct store_of<bf16> {
    template <class V> __host__ __device__ static bf16 get(V v) { return float_to_bf16((float)v); }
};
template <class TO, class V> __host__ __device__ inline TO to_store(V v) { return store_of<TO>::get(v); }

// Pointers to column blocks (each n x P, row-major, leading dimension P).
constexpr int MAXB = 64;
struct BlockPtrs {
    const void* p[MAXB];
};

constexpr int NT = 256;       // threads per workgroup of the streaming kernels
constexpr int MAXI = 24;      // register accumulators per thread in the dot kernels
constexpr int NWG_MAX = 1024; // workgroups of a streaming launch

// control block written by the per-step kernel and read by every kernel of a cycle
struct Ctl {
    int active;   // 1 while the cycle keeps stepping
    int meff;     // completed block steps of the current cycle
    int status;   // 0 ok, 1 Cholesky breakdown
    int pad;
};

inline int nwg_for(int64_t n, int P) {
    int64_t rows = NT / P;
    int64_t tiles = (n + rows - 1) / rows;
    int64_t g = tiles < NWG_MAX ? tiles : NWG_MAX;
    if (g >= 8) g -= g % 8;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------------------
// launchers (kernels.hip); every one enqueues on `st` and returns a hipError_t
// ---------------------------------------------------------------------------
template <class T>
struct Launch {
    using A = acc_t<T>;
    // W = (A Vin) Rinv; Vout = Vin Rinv (own rows); partial dots of [Q.., Vout]^H W
    static hipError_t spmm_dot(hipStream_t st, int P, int64_t n, const int* rp, const int* ci,
                               const T* av, const T* Vin, const A* Rinv, T* Vout, T* Wout,
                               const BlockPtrs& Q, int nq, int with_self, A* part, int nwg,
                               const Ctl* ctl);
    // sweep 1: W = (A Vin) Rinv, Vout = Vin Rinv (Rinv may be NULL = identity)
    static hipError_t spmm_rinv(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci,
                                const T* av, const T* Vin, const A* Rinv, T* Vout, T* Wout,
                                const Ctl* ctl);
    // W' = W - Q S (S optional) then W' = W' Rmul (optional); store W' (optional);
    // partials [Q^H W' (dot_q)] [W'^H W' (gram)]
    // kind: 1 = Arnoldi sweep 2 (k_proj_dot), 2 = Arnoldi sweep 3 (k_proj_gram), 0 = other (k_tsdot)
    static hipError_t update_dot(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q,
                                 int nq, const A* S, const A* Rmul, T* Wout, int dot_q, int gram,
                                 A* part, int nwg, const Ctl* ctl, int kind = 0);
    // out_o (+)= sum_i in_i coef[i][o]   (coef layout [nin][P][nout][P], FP64/complex128)
    template <class TO>
    static hipError_t combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin,
                              const BlockPtrs& out, int nout, const A* coef, int accumulate);
};

// reduce partials: out[o] = (add && o < nadd ? add[o] : 0) + sum_w part[w*nout + o]
// (nadd < 0: all outputs)
template <class A>
hipError_t reduce_partials(hipStream_t st, const A* part, int nwg, int nout, const A* add, A* out,
                           const Ctl* ctl, int nadd = -1);

// R = B - A X in FP64 (complex128); optional store of R narrowed to TR; per-WG
// partial sums [|r_b|^2 (P)] [|b_b|^2 (P)] into part (double)
template <class TA, class TR>
hipError_t residual(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const TA* av,
                    const TA* B, int64_t ldb, const TA* X, TR* Rout, double* part, int nwg);

// small kernels read a reduced P x P Gram matrix
// first CholQR pass of the start block; with nrhs < P (enlarged block) the
// enlarging columns are scaled to the residual's norm and Z1inv is D Z1^{-1}
template <class A>
hipError_t cholqr_first(hipStream_t st, int P, const A* gram, A* Z1, A* Z1inv, int nrhs, Ctl* ctl);
// second CholQR pass of the start block; g = E Z with only its first nrhs
// columns kept (nrhs < P: enlarged block, right-hand side E_1 F_0 e_1)
template <class A>
hipError_t cholqr_second(hipStream_t st, int P, const A* gram, const A* Z1, A* Rinv0, A* g, int m, int nrhs,
                         Ctl* ctl);
// columns c0 .. P-1 of the row-major n x P block Y <- SplitMix64 vectors in
// [-1, 1) (the enlarging vectors of a single right-hand side)
template <class T>
hipError_t fill_enlarging(hipStream_t st, T* Y, int64_t n, int P, int c0, uint64_t seed);
// S[r][c] = 0 for the columns c < ncols of a row-major rows x P matrix
template <class A>
hipError_t zero_cols(hipStream_t st, A* S, int rows, int P, int ncols);
// S1 non-null: `gram` is W'^H W' of the second pass and W''^H W'' = gram - S2^H S2
// with S2 = S - S1 (Pythagorean Gram of the stored block)
template <class A>
hipError_t step_small(hipStream_t st, int P, const A* gram, const A* S, const A* S1, int KP, int j, int m, A* H, A* F,
                      A* Rh, A* QH, A* g, A* RinvAll, double* rho, Ctl* ctl, double thresh);

// matrix-core versions of the three Arnoldi sweeps (real FP64/FP32 storage,
// P = 8 or 16); hipErrorNotSupported for other shapes.  nwg workgroups of
// 64-row tiles (mfma_nwg gives the default).  Each workgroup sweeps one
// contiguous range of row tiles; rev = true walks it from its end (FP64
// kernels), so that a sweep starts on the rows the previous one read last.
int mfma_nwg(int64_t n);
hipError_t i_minus(hipStream_t st, const double* M, double* out, int P);
// T is the arithmetic type (FP64 or FP32); TW, TQ and TO the storage types of
// the W blocks, the Q blocks and the output (T itself, or BF16 for basis
// blocks of the FP32 form).
// partial dots [Q_0 .. Q_{nq-1}]^T [W_0 .. W_{nw-1}] (no update), partial
// layout part[wg][w][c P + b]; at most 32 W columns, and then at most 9
// chunks of 16 Q columns, per launch (hipErrorNotSupported otherwise)
template <class T, class TW = T, class TQ = T>
hipError_t mfma_dot(hipStream_t st, int P, int64_t n, const BlockPtrs& W, int nw, const BlockPtrs& Q, int nq,
                    double* part, const Ctl* ctl, int nwg, bool rev = false);
// sweep 2: partial Q^T (W - Q S) and, with gram, (W - Q S)^T (W - Q S) after it
template <class T, class TQ = T>
hipError_t mfma_proj_dot(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S,
                         double* part, const Ctl* ctl, int nwg, bool gram = false, bool rev = false);
// sweep 3: W'' = W - Q S stored with its Gram partials, or with Rinv given,
// V = W'' Rinv stored (no Gram); with a control block it runs while the cycle
// is active and also for block step `step` if the cycle just stopped there
template <class T, class TQ = T, class TO = T>
hipError_t mfma_proj_gram(hipStream_t st, int P, int64_t n, const T* Win, const BlockPtrs& Q, int nq,
                          const double* S, TO* Wout, double* part, const Ctl* ctl, int nwg,
                          const double* Rinv = nullptr, int step = -1, bool rev = false);

// Sweeps 1a and 1b of a block step in one pass (real FP64, P = 8 or 16, at
// most 12 chunks of 16 columns in Q; hipErrorNotSupported otherwise):
// W = A Vin stored, and the partial first-pass dots [Q_0 .. Q_{nq-1}]^T W in
// part[wg][c P + w] for spmm_dot_nwg(P, n) workgroups.  Skipped while the
// cycle is inactive.
int spmm_dot_nwg(int P, int64_t n);
hipError_t spmm_dot_mfma(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const double* av,
                         const double* Vin, double* Wout, const BlockPtrs& Q, int nq, double* part, const Ctl* ctl);

// Sweep 1 of a block step with separate storage types: W = (A Vin) Rinv and
// Vout = Vin Rinv, or W = A Vin alone (Rinv and Vout NULL).  T is the type of
// the matrix values and of the arithmetic; TI, TV, TW those of Vin, Vout, W.
template <class T, class TI, class TV, class TW>
hipError_t spmm_block(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const T* av,
                      const TI* Vin, const acc_t<T>* Rinv, TV* Vout, TW* Wout, const Ctl* ctl);

// Y (+)= [in..] C on matrix cores (real FP64/FP32/BF16 inputs, FP64
// coefficients row-major (nin P) x (nout P)); the first `accumulate` output
// blocks are accumulated, the rest overwritten; hipErrorNotSupported for other
// shapes
template <class TI, class TO>
hipError_t mfma_combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                        const double* coef, int accumulate, int nwg);

hipError_t cast_values(hipStream_t st, const double* in, float* out, int64_t nnz);
// Block-CGS sweep of a one-column block (P = 1, real data, nq <= 32 blocks in
// Q, nwg workgroups): w' = w - Q s (S: nq FP64 coefficients, or null for no
// update); dot: partial Q^T w' (part[wg][nq]); otherwise w' stored in Wout
// and partial w'^T w' (part[wg][1]).  hipErrorNotSupported outside that range.
template <class T>
hipError_t narrow_sweep(hipStream_t st, int64_t n, const T* Win, const BlockPtrs& Q, int nq, const double* S, T* Wout,
                        double* part, int nwg, const Ctl* ctl, bool dot);

template <class TI, class TO>
hipError_t copy_block(hipStream_t st, int64_t n, int p, const TI* in, int64_t ldi, TO* out,
                      int64_t ldo, int zero_pad_to);

// The three block-CGS sweeps of complex128 blocks of P = 8 or 16 columns on
// the FP64 matrix cores, the blocks seen as real blocks of 2P interleaved
// (re, im) columns; nwg workgroups (mfma_nwg); at most cx_mfma_max_blocks(P,
// pip) blocks in Q (pip: the sweeps of the PIP order, second pass with the
// Gram of W', third pass normalising), hipErrorNotSupported otherwise.
// Partials are the real products part[wg][r 2P + s] of the 2q x 2P real view
// (q = nq P), which cx_reduce contracts into the complex q x P result.
int cx_mfma_max_blocks(int P, bool pip);
// partial Q^T W
hipError_t cx_dot(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, double* part,
                  const Ctl* ctl, int nwg, bool rev);
// W' = W - Q S (S complex q x P) and partial Q^T W', with gram followed by
// the partial real Gram of W' (2P x 2P, per-workgroup stride 4 q P + 4 P P);
// Sr (4 q P doubles) holds the real form of S (P = 8); Wtmp (n x P) receives
// W' for P = 16 with more than 10 blocks in Q (no Gram then)
hipError_t cx_proj_dot(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                       double* Sr, zd* Wtmp, double* part, const Ctl* ctl, int nwg, bool gram, bool rev);
// W'' = W - Q S stored in Wout with its partial real Gram (part[wg][r 2P + s],
// 2P x 2P); runs while the cycle is active and for block step `step` if it
// just stopped there
hipError_t cx_proj_gram(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                        double* Sr, zd* Wout, double* part, const Ctl* ctl, int nwg, int step);
// Y (+)= [in..] C for complex blocks (P = 8 or 16) on the FP64 matrix cores,
// C complex row-major (nin P) x (nout P), at most 64 real output columns; the
// first `accumulate` output blocks are accumulated
hipError_t cx_combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                      const zd* coef, int accumulate, int nwg);
// V = (W - Q S) R^{-1} stored in Vout (Rinv complex P x P); Sr holds
// 4 q P + 4 P P doubles (the real forms of S and R^{-1}, P = 8); runs while
// the cycle is active and for block step `step` if it just stopped there
hipError_t cx_proj_norm(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                        double* Sr, const zd* Rinv, zd* Vout, double* part, const Ctl* ctl, int nwg, int step,
                        bool rev);
// out = I - M for a complex P x P matrix (the update form of a right
// multiplication, W M = W - W (I - M))
hipError_t cx_i_minus(hipStream_t st, const zd* M, zd* out, int P);
// out (q x P) = add (or 0) + contraction of the summed real partials
// part[wg stride + off ..]
hipError_t cx_reduce_at(hipStream_t st, const double* part, int nwg, int64_t stride, int64_t off, int q, int P,
                        const zd* add, zd* out, const Ctl* ctl);
// the same with stride 4 q P and no offset
hipError_t cx_reduce(hipStream_t st, const double* part, int nwg, int q, int P, const zd* add, zd* out,
                     const Ctl* ctl);

// ---------------------------------------------------------------------------
// ILU(0) right preconditioning (ilu.hip).  The factors live in `lu`, an array
// with the CSR pattern (rp, ci) of A: strictly lower part of L (unit diagonal
// implied) and the upper part of U; diag[i] is the position of (i, i).  Every
// launch handles the rows rows[0 .. nrows) of one level; T is double or zd.
// ---------------------------------------------------------------------------
// numeric factorization of one level in place (lu starts as a copy of A's
// values; entries -1 of rows are padding); *err = 1 on a zero or non-finite
// pivot
template <class T>
hipError_t ilu0_level(hipStream_t st, const int* rows, int nrows, const int* rp, const int* ci, const int* diag,
                      T* lu, int* err);
// The whole triangular solve (lower: L y = in; upper: U x = in) in one launch,
// rows taken in level order by the ticket counter `tick` and every entry of
// `out` waited for by value: `ord` (npad entries) lists the rows level by
// level, each level padded with -1 to a multiple of 256 / P entries; `out`
// must hold PENDING everywhere and *tick must be 0.  The launch re-arms
// `rearm` (its entries set to PENDING after `in` is read, so in may be rearm)
// and *tick_next = 0 for the next solve; *err = 1 if a bounded wait expired
// (the row then holds a NaN).  Skipped while the cycle is inactive.
template <class T>
hipError_t trsv_flow(hipStream_t st, int P, bool lower, int64_t npad, const int* ord, const int* rp, const int* ci,
                     const int* diag, const T* lu, const T* in, T* out, T* rearm, unsigned* tick, unsigned* tick_next,
                     int* err, const Ctl* ctl);
// count entries of y set to PENDING (the initial state of the two solve blocks)
template <class T>
hipError_t fill_pending(hipStream_t st, int64_t count, T* y);
// *diff = 1 where the CSR patterns (rpa, cia) and (rpb, cib) differ (same n, nnz)
hipError_t pattern_diff(hipStream_t st, int64_t n, int64_t nnz, const int* rpa, const int* cia, const int* rpb,
                        const int* cib, int* diff);
// out = in M row by row (M P x P, row-major); skipped while the cycle is inactive
template <class T>
hipError_t rows_times(hipStream_t st, int P, int64_t n, const T* in, const acc_t<T>* M, T* out, const Ctl* ctl);

}  // namespace bgcr
