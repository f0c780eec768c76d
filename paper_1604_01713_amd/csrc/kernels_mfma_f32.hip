// FP32 instantiations of the matrix-core Arnoldi sweeps (inner cycles of the
// mixed-precision solver); Gram matrices are still accumulated in FP64.
#include "mfma_sweeps.h"

namespace bgcr {

template hipError_t mfma_dot<float>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int, double*,
                                    const Ctl*, int, bool);
template hipError_t mfma_proj_dot<float>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                          const double*, double*, const Ctl*, int, bool, bool);
template hipError_t mfma_proj_gram<float>(hipStream_t, int, int64_t, const float*, const BlockPtrs&, int,
                                           const double*, float*, double*, const Ctl*, int, const double*,
                                           int, bool);

template hipError_t mfma_combine<float, float>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&,
                                                  int, const double*, int, int);
template hipError_t mfma_combine<float, double>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&,
                                                  int, const double*, int, int);

}  // namespace bgcr
