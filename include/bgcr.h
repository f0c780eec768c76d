/*
 * bgcr.h -- C ABI of the MI355X block GCRO-DR library (libbgcr.so).
 *
 * Block GCRO-DR (block recycled GMRES, Parks, Soodhalter and Szyld, Algorithm 1)
 * solves a sequence of non-Hermitian sparse systems A^[i] X = B^[i] with p
 * right-hand sides (Section 1, eq. (1.1)), keeping a recycled pair (U, C) with
 * A U = C and orthonormal C on the device between calls (Algorithm 1, last line).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (memory on the GPU the library runs
 *     on) unless the comment says "host".  Sizes are in elements.
 *   - Dense blocks are row-major n x p with a leading dimension ld >= p
 *     (element (i, j) at ptr[i*ld + j]).  Complex data (BGCR_C128) is
 *     interleaved (re, im) doubles.
 *   - Sparse matrices are 0-based CSR with int32 row_ptr[n+1] and col_idx[nnz];
 *     values are double (BGCR_F64) or interleaved complex double (BGCR_C128).
 *     The indices are 32-bit only: a matrix with nnz >= 2^31 is rejected with
 *     BGCR_ERR_INVALID before anything is enqueued.
 *   - The caller owns every array it passes in; the library never frees them
 *     and keeps no pointer to them after the call returns.
 *   - Every function returns a status code (BGCR_OK = 0, see bgcr_status);
 *     no C++ exception crosses this boundary.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the legacy
 *     default stream).  Calls on different sequences may run concurrently from
 *     different host threads; one sequence is not re-entrant.
 */
#ifndef BGCR_H
#define BGCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BGCR_OK = 0,
    BGCR_NOT_CONVERGED = 1,        /* max_cycles reached; X holds the last iterate */
    BGCR_BREAKDOWN_DEFLATED = 2,   /* converged (X valid, as for BGCR_OK), and on the way
                                      at least one block was numerically rank deficient
                                      and handled: a start block rebuilt from its
                                      independent columns and seeded vectors, or a
                                      cycle ended at a block-step breakdown (count in
                                      bgcr_stats.deflations) */
    BGCR_ERR_INVALID = -1,         /* NULL/ill-sized argument, n or p mismatch, tol <= 0 */
    BGCR_ERR_NOMEM = -2,           /* device allocation failed */
    BGCR_ERR_HIP = -3,             /* HIP runtime error, including no visible device */
    BGCR_ERR_NONFINITE = -4,       /* NaN/Inf in A, B or X0, or produced during the solve */
    BGCR_ERR_NUMERICAL = -5        /* rank-deficient Krylov block (Cholesky breakdown)
                                      or eigensolver failure */
} bgcr_status;

typedef enum { BGCR_F64 = 0, BGCR_C128 = 1 } bgcr_dtype;

typedef enum {
    BGCR_PLAIN_FP64 = 0,           /* every step in FP64 (complex128 for BGCR_C128) */
    BGCR_MIXED_FP32 = 1,           /* FP32 SpMM/basis/BCGS2 cycles inside an FP64
                                      iterative-refinement loop (real data only) */
    BGCR_MIXED_FP32_BF16 = 2       /* as BGCR_MIXED_FP32 with the basis blocks (V, U, C)
                                      stored in BF16 (round to nearest even) and widened
                                      to FP32 on every load; W, R, Gram, LSQ, eigenproblem
                                      and the solution as in BGCR_MIXED_FP32.  Real data,
                                      p = 8 or 16, 2 * ceil((k+1)/p) * p <= 64; otherwise
                                      bgcr_create_sequence returns BGCR_ERR_INVALID */
} bgcr_precision;

typedef enum {
    BGCR_PRECOND_NONE = 0,
    BGCR_PRECOND_ILU0 = 1          /* right preconditioning with the zero-fill incomplete LU
                                      factorization of each system's A (the preconditioner of
                                      the paper's experiments, Sections 6.1 and 6.2): the
                                      cycles run on A M^{-1}, M = L U with L unit lower and U
                                      upper triangular on the pattern of A and (L U)_ij = A_ij
                                      there; X stays the unpreconditioned unknown, the
                                      stopping test uses B - A X, and the recycled U lives in
                                      the preconditioned variable.  Every row of A needs its
                                      diagonal entry and sorted column indices (else
                                      BGCR_ERR_INVALID at bgcr_solve); a zero pivot gives
                                      BGCR_ERR_NUMERICAL.  Plain FP64 (real or complex) with
                                      block_size 0 or p and no hybrid; otherwise
                                      bgcr_create_sequence returns BGCR_ERR_INVALID */
} bgcr_precond;

typedef struct bgcr_sequence bgcr_sequence;   /* opaque; owns U, C and workspaces */

typedef struct {
    int32_t p;               /* number of right-hand sides = block size: 1, 2, 4, 8 or 16 */
    int32_t m;               /* block Arnoldi steps per cycle (1..64); with KB =
                                ceil((k+1)/L) blocks of the recycled space (ceil(k/L)
                                for complex data, L the block size), 2 KB + m + 1 <= 64:
                                the refresh combines [U, C, V_1 .. V_{m+1}] in one
                                launch.  Otherwise BGCR_ERR_INVALID */
    int32_t k;               /* recycled dimension (0..128); with real data k+1 columns
                                are kept when a conjugate pair straddles the cut */
    int32_t dtype;           /* bgcr_dtype */
    int32_t precision;       /* bgcr_precision */
    int32_t max_cycles;      /* restart cycles per solve before BGCR_NOT_CONVERGED (>= 1) */
    int32_t select_largest;  /* 0: keep harmonic Ritz values of smallest modulus
                                (Section 4.1 default); 1: largest */
    int32_t block_size;      /* block size L of the Krylov basis: 0 or p for L = p.
                                With p = 1, L in {2, 4, 8, 16} enlarges the block
                                (Section 3.1, eq. 1rhs-block-gmres-min): every cycle
                                starts from [r, Z], Z the same L - 1 vectors drawn by
                                SplitMix64 (entry (i, c) from the counter
                                i + 2^40 c, mapped to [-1, 1)), and minimises the
                                single residual; U, C and the basis are n x L blocks,
                                B and X stay n x 1.  Other values: BGCR_ERR_INVALID */
    int32_t enlarge_cycles;  /* hybrid of Section 4.1.3 (needs an enlarged block,
                                block_size > p = 1): the first enlarge_cycles
                                restart cycles of the sequence, counted over all its
                                solves, use block size L and every later cycle is
                                non-block GCRO-DR (L = 1); at the switch the
                                recycled U is handed to the L = 1 basis and imported
                                there (A U = C S).  0: every cycle uses L.  Not with
                                BGCR_MIXED_FP32_BF16; negative: BGCR_ERR_INVALID */
    int32_t ritz_vectors;    /* recycled space: 0 harmonic Ritz vectors (Section 4.1.2);
                                1 Ritz vectors (Section 4.1.3): the first cycle takes
                                eigenvectors of the square block Hessenberg H_m, later
                                cycles the Galerkin pencil on U + K_m,
                                (What^H A What) t = theta (What^H What) t with
                                What = [U D, V_1 .. V_m].  The selection by modulus
                                follows select_largest.  Other values: BGCR_ERR_INVALID */
    int32_t precond;         /* bgcr_precond.  The factorization of each system is computed
                                on the device at every bgcr_solve; the level schedule of its
                                triangular solves is computed on the host when the pattern
                                differs from the last one the sequence analysed */
} bgcr_params;

typedef struct {
    int64_t n;               /* rows = columns */
    int64_t nnz;
    const int32_t* row_ptr;  /* device, n+1 entries */
    const int32_t* col_idx;  /* device, nnz entries */
    const void* values;      /* device, nnz entries (double or interleaved complex double) */
} bgcr_csr;

typedef struct {
    int32_t status;          /* same as the return code of bgcr_solve */
    int32_t cycles;          /* restart cycles, including the first-system block GMRES cycle */
    int32_t block_steps;     /* block Arnoldi steps over all cycles */
    int32_t spmm_calls;      /* block SpMMs (n x p) with A, any precision */
    double rel_res;          /* ||B - A X||_F / ||B||_F at return (FP64) */
    double rel_res_max_col;  /* max_j ||b_j - A x_j|| / ||b_j|| at return */
    double seconds;          /* host wall time of the call */
    double alg_bytes;        /* algorithmic HBM bytes of the block Arnoldi sweeps executed */
    int32_t k_eff;           /* columns of the recycled space stored at return */
    int32_t refine_steps;    /* FP64 refinement steps (BGCR_MIXED_FP32), else 0 */
    int32_t deflations;      /* rank-deficient blocks handled in this call: start blocks
                                rebuilt plus cycles ended at a block-step breakdown */
} bgcr_stats;

/* Create a sequence for systems of order n (Algorithm 1 parameters m, k and
 * block size p in prm).  Allocates the recycled pair, the block Arnoldi basis
 * and every workspace on the current HIP device (size: bgcr_footprint_bytes).
 * hip_stream: a hipStream_t all work of this sequence is enqueued on.
 * out: host pointer receiving the handle.  Errors: INVALID, NOMEM, HIP. */
int bgcr_create_sequence(const bgcr_params* prm, int64_t n, void* hip_stream,
                         bgcr_sequence** out);

/* Solve A X = B for the next system of the sequence (Algorithm 1).
 * A: CSR of order n (device arrays; may differ at every call, Section 1).
 * B: n x p right-hand sides with leading dimension ldb (read only).
 * X: n x p, on entry the initial guess X0, on return the solution (ldx).
 * tol: relative tolerance, stop when ||B - A X||_F <= tol ||B||_F.
 * st: host pointer or NULL; receives the statistics of this call.
 * The first call takes the no-U branch of Algorithm 1 (one block GMRES cycle,
 * then harmonic Ritz selection); later calls import the stored U (A U = C S).
 * Blocks the calling thread until the result is in X.
 * Returns OK, BREAKDOWN_DEFLATED (converged after handling a rank-deficient
 * block), NOT_CONVERGED (X holds the last iterate), INVALID (including
 * A->nnz >= 2^31), HIP, NONFINITE (NaN or Inf in A, B or X0, or produced
 * during the solve) or NUMERICAL. */
int bgcr_solve(bgcr_sequence* s, const bgcr_csr* A, const void* B, int64_t ldb,
               void* X, int64_t ldx, double tol, bgcr_stats* st);

/* Free U, C and every workspace of the sequence.  NULL is a no-op. */
int bgcr_release(bgcr_sequence* s);

/* Device bytes a sequence with these parameters allocates for order n and a
 * matrix with nnz nonzeros (used for admission by HBM budget).  0 if prm is
 * invalid. */
size_t bgcr_footprint_bytes(const bgcr_params* prm, int64_t n, int64_t nnz);

/* Number of recycled columns currently stored (0 before the first solve). */
int bgcr_recycle_dim(const bgcr_sequence* s, int32_t* k_eff);

/* Copy the stored recycled pair out (Algorithm 1: U is kept for the next
 * call).  U_out and C_out: device, n x k_eff row-major with leading dimension
 * ld >= k_eff, in the sequence's basis precision widened to FP64 (complex128
 * for BGCR_C128).  Either pointer may be NULL. */
int bgcr_get_recycle(const bgcr_sequence* s, void* U_out, void* C_out, int64_t ld);

/* Replace the stored recycled space by the k_in columns of U_in (device,
 * n x k_in, leading dimension ld, FP64 or complex128): the optional U input of
 * Algorithm 1.  C is formed at the next solve by A U = C S.  k_in <= k+1. */
int bgcr_set_recycle(bgcr_sequence* s, const void* U_in, int64_t ld, int32_t k_in);

/* Per-cycle log of the last solve (host arrays of capacity cap): block steps
 * of each cycle and the true relative residual ||B - A X||_F/||B||_F after it.
 * *count receives the number of cycles (may exceed cap; only cap are written). */
int bgcr_get_cycle_log(const bgcr_sequence* s, int32_t* steps, double* rel_res,
                       int32_t cap, int32_t* count);

/* Standalone block SpMM W = A V (the dominant kernel of the cycle, Section 6.3):
 * V, W: device, n x p row-major, leading dimension p.  dtype BGCR_F64 or
 * BGCR_C128, p in {1, 2, 4, 8, 16}.  hip_stream may be NULL. */
int bgcr_spmm(const bgcr_csr* A, int32_t dtype, int32_t p, const void* V, void* W,
              void* hip_stream);

/* Projected operator of the data-movement study (Section 6.3), real FP64:
 * W = (I - C C^T) A V, where C has orthonormal columns.
 *   A: CSR of order n (device arrays).
 *   V, W: device, n x p row-major (leading dimension p), p in {1, 2, 4, 8, 16}; W
 *         is overwritten and must not alias V.
 *   C: device, kc >= 0 blocks of n x p row-major stored one after the other (block
 *      b at C + b n p); zero columns are allowed as padding; must not overlap W.
 *   variant: 0 two passes of block classical Gram-Schmidt over all of C (each pass:
 *            all dots C^T W, then W -= C S), the multi-pass CGS of Section 6.3;
 *            1 block modified Gram-Schmidt, one pass, one block of C after the
 *            other (s_b = C_b^T W, W -= C_b s_b); with p = 1 it is the
 *            column-wise MGS of Section 6.3.
 *   work: device scratch of at least bgcr_apply_projected_work_bytes(n, p, kc) bytes
 *         (partials and coefficients; owned by the caller, contents ignored).
 * Enqueued on hip_stream (may be NULL); returns once enqueued.  Errors: INVALID
 * (NULL pointers, unsupported p or variant, kc < 0, short workspace, nnz < 0), HIP. */
int bgcr_apply_projected(const bgcr_csr* A, int32_t p, int32_t kc, const double* C,
                         const double* V, double* W, int32_t variant, void* work,
                         size_t work_bytes, void* hip_stream);

/* Workspace bytes bgcr_apply_projected needs for (n, p, kc); 0 for invalid p or
 * kc < 0. */
size_t bgcr_apply_projected_work_bytes(int64_t n, int32_t p, int32_t kc);

/* Size of the library's own device workspace used by
 * bgcr_apply_projected_noalloc (20 MiB; each GPU the library runs on holds one
 * until the process ends). */
#define BGCR_NOALLOC_SCRATCH_BYTES (20u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as bgcr_apply_projected, with the same kernels and results, but
 * the workspace is a device array inside the library, so no call allocates
 * (no hipMalloc, hipFree or allocating library routine).
 *   A, p, kc, C, V, W, variant, hip_stream: as for bgcr_apply_projected; the
 *   caller still owns and passes the inputs and the output.
 * Limit: bgcr_apply_projected_work_bytes(n, p, kc) must not exceed
 * BGCR_NOALLOC_SCRATCH_BYTES (p = 16: kc <= 1536 blocks; p <= 8: kc <= 32250),
 * else BGCR_ERR_INVALID before anything is enqueued.
 * Every call on one GPU shares that GPU's workspace, which keeps the last
 * call's contents (nothing in it needs to start at zero): calls that overlap on
 * one GPU, from several streams or threads, race and give undefined results.
 * Errors: INVALID (as bgcr_apply_projected, or the size limit), HIP (no device,
 * or the workspace address could not be looked up). */
int bgcr_apply_projected_noalloc(const bgcr_csr* A, int32_t p, int32_t kc, const double* C,
                                 const double* V, double* W, int32_t variant, void* hip_stream);

/* Kernel classes of the per-kernel profile. */
typedef enum {
    BGCR_K_ARN_SPMM = 0,     /* Arnoldi sweep 1a: W = A V_j with V_j = W'' R^{-1} */
    BGCR_K_ARN_DOT = 1,      /* Arnoldi sweep 1b: first block-CGS dots [C V_1..V_j]^H W */
    BGCR_K_PROJ_DOT = 2,     /* Arnoldi sweep 2: second block-CGS pass */
    BGCR_K_PROJ_GRAM = 3,    /* Arnoldi sweep 3: W'' = W - Q S and its Gram */
    BGCR_K_SMALL = 4,        /* partial reductions, Cholesky, block-Householder LSQ */
    BGCR_K_COMBINE = 5,      /* basis updates: solution, residual, recycle refresh */
    BGCR_K_RESIDUAL = 6,     /* FP64 true residual B - A X */
    BGCR_K_TSDOT = 7,        /* other tall-skinny products (CholQR of R, recycle dots) */
    BGCR_K_SPMM = 8,         /* plain block SpMM (recycle import A U) */
    BGCR_K_HOST = 9,         /* host: small dense algebra of a cycle (wall clock, includes BGCR_K_HOST_EIG) */
    BGCR_K_HOST_EIG = 10,    /* host: harmonic-Ritz eigenproblem (wall clock) */
    BGCR_K_PRECOND = 11,     /* triangular solves of M^{-1} (ILU(0) preconditioning) */
    BGCR_K_ILU = 12,         /* ILU(0): pattern check and analysis, numeric factorization */
    BGCR_K_ARN_SPMM_DOT = 13,/* Arnoldi sweeps 1a and 1b in one pass: W = A V_j and the first
                                block-CGS dots (FP64 on matrix cores, from the second step) */
    BGCR_K_NCLASS = 14
} bgcr_kernel_class;

/* Turn per-kernel timing on (1) or off (0) and reset the counters.  When on,
 * every launch of the sequence is bracketed by HIP events on its stream and
 * its algorithmic HBM bytes are counted (block steps skipped after an early
 * exit of a cycle are not counted). */
int bgcr_set_profiling(bgcr_sequence* s, int on);

/* Accumulated profile since the last bgcr_set_profiling: per kernel class,
 * total milliseconds, algorithmic bytes and launches (host arrays of nclass
 * entries, any may be NULL). */
int bgcr_get_profile(const bgcr_sequence* s, double* ms, double* bytes, int64_t* launches,
                     int32_t nclass);

/* Measurement aid (not a step of the method): the streaming rate the memory
 * system sustains for a mix of read and written FP64 blocks, with the row-tile
 * schedule of the block-step sweeps (XCD-aware contiguous row spans, 16-byte
 * accesses).  Every out[o][i] = sum over b of in[b][i], for i < count.
 *   in:    host array of nin device pointers (1 <= nin <= 16), 16-byte aligned.
 *   out:   host array of nout device pointers (0 <= nout <= 4), 16-byte aligned,
 *          not aliasing any input; may be NULL when nout is 0.
 *   count: doubles per block, even (0: nothing is launched).
 *   nwg:   workgroups (0: 512, the grid of the sweeps); capped at the tile count.
 * Asynchronous on hip_stream (may be NULL).  INVALID for bad arguments, HIP
 * when the launch fails. */
int bgcr_stream_probe(const double* const* in, int32_t nin, double* const* out, int32_t nout,
                      int64_t count, int32_t nwg, void* hip_stream);

/* Human-readable text of a status code (static storage). */
const char* bgcr_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
