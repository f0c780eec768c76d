// FP64 instantiations of the matrix-core Arnoldi sweeps, the block SpMM fused
// with the first-pass dots, and the small helpers shared by both storage
// types.
#include "mfma_sweeps.h"
#include "spmm_sweep.h"

namespace bgcr {

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

// two resident workgroups per CU, 256 CUs: one wave of workgroups
int mfma_nwg(int64_t n) {
    constexpr int64_t kMax = 512;
    const int64_t tiles = (n + mx::MROWS - 1) / mx::MROWS;
    int64_t g = tiles < kMax ? tiles : kMax;
    if (g >= 8) g -= g % 8;
    return (int)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// Sweeps 1a and 1b of a block step in one pass over the rows: W = A V (the
// row layout of the block SpMM, stored) and the partial first-pass dots
// [Q_0 .. Q_{nq-1}]^T W on matrix cores, in the partial layout of the dot
// sweep with one W block (part[wg][c P + w], c < nq P).  Per tile of ROWS
// rows: the tile's Q rows are requested first, so that they stream in while
// the SpMM gathers V; the W tile is staged in LDS (rows past n as zeros) and
// read back as the A operand (W[row][w], w = l % 16; lanes w >= P repeat
// column w % P and feed partial rows that are never written).  Each wave
// takes ROWS / 4 rows of the tile, KS = ROWS / 16 slices of 4: exactly the
// rows its own lanes computed in the SpMM layout (P / 2 lanes per row), so
// the staging is wave-private and the loop has no workgroup barrier.  Tiles
// follow the SpMM's XCD-local order (the stencil neighbours stay in the
// XCD's L2).
// ---------------------------------------------------------------------------
template <int P, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NC <= 8 ? 2 : 1))) void k_spmm_dot_mfma(int64_t n, int64_t nnz, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const double* __restrict__ av,
                                                       const double* __restrict__ Vin, double* __restrict__ Wout,
                                                       BlockPtrs Q, int nq, double* __restrict__ part,
                                                       const Ctl* ctl) {
    using M = mx::MX<double>;
    constexpr int C = 2, LPR = P / C, ROWS = 256 / LPR, WR = ROWS / 4, KS = WR / 4;
    static_assert(KS >= 1 && WR % 4 == 0, "whole 4-row slices per wave");
    static_assert(WR * LPR == 64, "a wave's SpMM rows are the rows of its dot slices");
    if (ctl && ctl->active == 0) return;
    __shared__ double Wt[ROWS * P];
    __shared__ double red[1024];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, r = t / LPR, prt = t % LPR, c0 = prt * C;
    const int q = nq * P;
    const double* qp[NC];
    mx::rc_pointers<double, P, NC>(qp, Q, nq, lane);
    M::acc acc[1][NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[0][ch] = M::acc{0, 0, 0, 0};
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    int64_t first, step, end;
    sp::xcd_tiles(ntiles, first, step, end);
    const int64_t nzl = nnz - 1;
    const int wcol = (lane & 15) & (P - 1);
    for (int64_t tile = first; tile < end; tile += step) {
        const int64_t rb = tile * ROWS + wave * WR;
        // Q streams through once: non-temporal loads, so that the L2 keeps the
        // gathered neighbour rows of V
        double qv[KS][NC];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int64_t off = mx::clamp_row(rb + 4 * ks + (lane >> 4), n) * P;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) qv[ks][ch] = __builtin_nontemporal_load(qp[ch] + off);
        }
        const int64_t row = tile * ROWS + r;
        const int64_t rowc[1] = {mx::clamp_row(row, n)};
        double raw[1][C];
        sp::row_product<double, double, P, C, LPR == 4, 1>(raw, rp, ci, av, Vin, rowc, prt, c0, nzl);
        if (row < n) sp::store_as<double, double, C, P>(Wout + row * P + c0, raw[0]);
#pragma unroll
        for (int j = 0; j < C; ++j) Wt[r * P + c0 + j] = row < n ? raw[0][j] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const double a = Wt[(wave * WR + 4 * ks + (lane >> 4)) * P + wcol];
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) acc[0][ch] = M::mma(a, qv[ks][ch], acc[0][ch]);
        }
        // the next tile's staging overwrites this wave's rows only after every
        // lane has read them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    mx::write_dot_partials<double, P, 1, NC>(acc, q, 1, red, part, blockIdx.x);
}

// two resident workgroups per CU (two waves per SIMD): one wave of workgroups
int spmm_dot_nwg(int P, int64_t n) {
    const int64_t rows = 256 / (P / 2);
    const int64_t tiles = (n + rows - 1) / rows;
    int64_t g = tiles < 512 ? tiles : 512;
    if (g >= 8) g -= g % 8;
    return (int)(g < 1 ? 1 : g);
}

hipError_t spmm_dot_mfma(hipStream_t st, int P, int64_t n, int64_t nnz, const int* rp, const int* ci, const double* av,
                         const double* Vin, double* Wout, const BlockPtrs& Q, int nq, double* part, const Ctl* ctl) {
    const int nc = (nq * P + 15) / 16;
    const int g = spmm_dot_nwg(P, n);
#define BGCR_SD(PP, NC)                                                                                              \
    case NC:                                                                                                         \
        hipLaunchKernelGGL((k_spmm_dot_mfma<PP, NC>), dim3(g), dim3(256), 0, st, n, nnz, rp, ci, av, Vin, Wout, Q,  \
                           nq, part, ctl);                                                                           \
        return hipGetLastError();
#define BGCR_SD_P(PP)                                                                                                \
    switch (nc) {                                                                                                    \
        BGCR_SD(PP, 1) BGCR_SD(PP, 2) BGCR_SD(PP, 3) BGCR_SD(PP, 4) BGCR_SD(PP, 5) BGCR_SD(PP, 6) BGCR_SD(PP, 7)      \
        BGCR_SD(PP, 8) BGCR_SD(PP, 9) BGCR_SD(PP, 10) BGCR_SD(PP, 11) BGCR_SD(PP, 12)                               \
        default: return hipErrorNotSupported;                                                                        \
    }
    if (P == 8) BGCR_SD_P(8)
    if (P == 16) BGCR_SD_P(16)
#undef BGCR_SD_P
#undef BGCR_SD
    return hipErrorNotSupported;
}

template hipError_t mfma_dot<double>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int, double*,
                                     const Ctl*, int, bool);
template hipError_t mfma_proj_dot<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                          const double*, double*, const Ctl*, int, bool, bool);
template hipError_t mfma_proj_gram<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                           const double*, double*, double*, const Ctl*, int, const double*,
                                           int, bool);

template hipError_t mfma_combine<double, double>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&,
                                                  int, const double*, int, int);

}  // namespace bgcr
