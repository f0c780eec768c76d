// Instantiations for the FP32 form with BF16 basis storage: the Krylov basis
// V and the recycle pair (U, C) are stored in BF16, W, R and the
// normalised start block in FP32; arithmetic is FP32 (Gram matrices and
// combination coefficients FP64).
#include "mfma_sweeps.h"
#include "spmm_sweep.h"

namespace bgcr {

// [C V_1 .. V_j]^T W with W in FP32 (Arnoldi sweep 1b, C^T R)
template hipError_t mfma_dot<float, float, bf16>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&,
                                                 int, double*, const Ctl*, int, bool);
// dots of basis blocks with basis blocks (Gram of C, refresh dots against U)
template hipError_t mfma_dot<float, bf16, bf16>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&,
                                                int, double*, const Ctl*, int, bool);
template hipError_t mfma_proj_dot<float, bf16>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                               const double*, double*, const Ctl*, int, bool, bool);
template hipError_t mfma_proj_gram<float, bf16, bf16>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                                      const double*, bf16*, double*, const Ctl*, int, const double*,
                                                      int, bool);

// R - C T with C in BF16 (enlarged start block projected against C)
template hipError_t mfma_proj_gram<float, bf16, float>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                                       const double*, float*, double*, const Ctl*, int, const double*,
                                                       int, bool);

template hipError_t mfma_combine<bf16, double>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int,
                                               const double*, int, int);
template hipError_t mfma_combine<bf16, float>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int,
                                              const double*, int, int);
template hipError_t mfma_combine<bf16, bf16>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int,
                                             const double*, int, int);

// SpMM: first step (FP32 start block -> BF16 V_1), later steps (BF16 V_j),
// and A U of the recycle import (BF16 -> BF16)
template hipError_t spmm_block<float, float, bf16, float>(hipStream_t, int, int64_t, int64_t, const int*, const int*,
                                                          const float*, const float*, const double*, bf16*, float*,
                                                          const Ctl*);
template hipError_t spmm_block<float, bf16, bf16, float>(hipStream_t, int, int64_t, int64_t, const int*, const int*,
                                                         const float*, const bf16*, const double*, bf16*, float*,
                                                         const Ctl*);
template hipError_t spmm_block<float, bf16, bf16, bf16>(hipStream_t, int, int64_t, int64_t, const int*, const int*,
                                                        const float*, const bf16*, const double*, bf16*, bf16*,
                                                        const Ctl*);

}  // namespace bgcr
