// FP64 instantiations of the matrix-core Arnoldi sweeps, and the small
// helpers shared by both storage types.
#include "mfma_sweeps.h"

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
