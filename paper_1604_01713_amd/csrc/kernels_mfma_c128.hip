// complex128 block-CGS sweeps on the FP64 matrix cores (real views of the
// interleaved blocks; the mapping is described in cplx_sweeps.h)
#include "cplx_sweeps.h"

namespace bgcr {

// the 16-column real sweeps are instantiated with the other FP64 kernels
extern template hipError_t mfma_dot<double>(hipStream_t, int, int64_t, const BlockPtrs&, int, const BlockPtrs&, int,
                                            double*, const Ctl*, int, bool);
extern template hipError_t mfma_proj_dot<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                                 const double*, double*, const Ctl*, int, bool, bool);
extern template hipError_t mfma_proj_gram<double>(hipStream_t, int, int64_t, const double*, const BlockPtrs&, int,
                                                  const double*, double*, double*, const Ctl*, int, const double*,
                                                  int, bool);

int cx_mfma_max_blocks(int P, bool pip) {
    // P = 8: the 16-column real sweeps (their second pass holds at most 14
    // chunks of Q in LDS); P = 16: the 32-column sweeps, dispatched up to 12,
    // the fused second pass (which the PIP order needs) up to 10
    return P == 8 ? 14 : (P == 16 ? (pip ? 10 : 12) : 0);
}

static hipError_t expand(hipStream_t st, const zd* S, int q, int P, double* Sr, const Ctl* ctl) {
    hipLaunchKernelGGL(mx::k_cx_expand, dim3((q * P + 255) / 256), dim3(256), 0, st, S, q, P, Sr, ctl);
    return hipGetLastError();
}

hipError_t cx_dot(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, double* part,
                  const Ctl* ctl, int nwg, bool rev) {
    if (nq < 1 || nq > cx_mfma_max_blocks(P, false)) return hipErrorNotSupported;
    if (P == 8) {
        BlockPtrs Wp{};
        Wp.p[0] = W;
        return mfma_dot<double>(st, 16, n, Wp, 1, Q, nq, part, ctl, nwg, rev);
    }
    return mx::launch_dot_wide(st, n, (const double*)W, Q, nq, part, nwg, ctl, rev);
}

hipError_t cx_proj_dot(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                       double* Sr, zd* Wtmp, double* part, const Ctl* ctl, int nwg, bool gram, bool rev) {
    if (nq < 1 || nq > cx_mfma_max_blocks(P, gram)) return hipErrorNotSupported;
    if (P == 8) {
        const hipError_t e = expand(st, S, nq * P, P, Sr, ctl);
        if (e != hipSuccess) return e;
        return mfma_proj_dot<double>(st, 16, n, (const double*)W, Q, nq, Sr, part, ctl, nwg, gram, rev);
    }
    // one fused sweep up to 10 blocks in Q; beyond, W' is stored and dotted
    // in a second sweep (no Gram)
    const hipError_t f = gram ? mx::launch_proj_dot_wide<true>(st, n, (const double*)W, Q, nq, S, part, nwg, ctl, rev)
                              : mx::launch_proj_dot_wide<false>(st, n, (const double*)W, Q, nq, S, part, nwg, ctl, rev);
    if (f != hipErrorNotSupported || gram) return f;
    const hipError_t e = mx::launch_update_wide_t<false>(st, n, (const double*)W, Q, nq, S, (double*)Wtmp, nullptr,
                                                         nwg, ctl, -1, false);
    if (e != hipSuccess) return e;
    return mx::launch_dot_wide(st, n, (const double*)Wtmp, Q, nq, part, nwg, ctl, true);
}

hipError_t cx_proj_gram(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                        double* Sr, zd* Wout, double* part, const Ctl* ctl, int nwg, int step) {
    if (nq < 1 || nq > cx_mfma_max_blocks(P, false)) return hipErrorNotSupported;
    if (P == 8) {
        const hipError_t e = expand(st, S, nq * P, P, Sr, ctl);
        if (e != hipSuccess) return e;
        return mfma_proj_gram<double>(st, 16, n, (const double*)W, Q, nq, Sr, (double*)Wout, part, ctl, nwg, nullptr,
                                      step, false);
    }
    return mx::launch_update_wide_t<true>(st, n, (const double*)W, Q, nq, S, (double*)Wout, part, nwg, ctl, step,
                                          false);
}

hipError_t cx_proj_norm(hipStream_t st, int P, int64_t n, const zd* W, const BlockPtrs& Q, int nq, const zd* S,
                        double* Sr, const zd* Rinv, zd* Vout, double* part, const Ctl* ctl, int nwg, int step,
                        bool rev) {
    if (nq < 1 || nq > cx_mfma_max_blocks(P, true)) return hipErrorNotSupported;
    if (P == 8) {
        // S and R^{-1} in real form: S_r, then the 16 x 16 R^{-1}_r after it
        // (expanded whatever the control block says: the sweep also runs
        // after the step that stopped the cycle, to store its V_{j+1})
        double* Rr = Sr + (size_t)4 * nq * P * P;
        hipError_t e = expand(st, S, nq * P, P, Sr, nullptr);
        if (e == hipSuccess) e = expand(st, Rinv, P, P, Rr, nullptr);
        if (e != hipSuccess) return e;
        return mfma_proj_gram<double>(st, 16, n, (const double*)W, Q, nq, Sr, (double*)Vout, part, ctl, nwg, Rr, step,
                                      rev);
    }
    return mx::launch_update_wide_t<false, true>(st, n, (const double*)W, Q, nq, S, (double*)Vout, nullptr, nwg, ctl,
                                                 step, rev, Rinv);
}

hipError_t cx_combine(hipStream_t st, int P, int64_t n, const BlockPtrs& in, int nin, const BlockPtrs& out, int nout,
                      const zd* coef, int accumulate, int nwg) {
    if (P == 8) return mx::launch_combine_cx<16>(st, n, in, nin, out, nout, (const double*)coef, accumulate, nwg);
    if (P == 16) return mx::launch_combine_cx<32>(st, n, in, nin, out, nout, (const double*)coef, accumulate, nwg);
    return hipErrorNotSupported;
}

__global__ void k_cx_i_minus(const zd* __restrict__ M, zd* __restrict__ out, int P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P * P) out[e] = zd{((e / P) == (e % P) ? 1.0 : 0.0) - M[e].x, -M[e].y};
}

hipError_t cx_i_minus(hipStream_t st, const zd* M, zd* out, int P) {
    hipLaunchKernelGGL(k_cx_i_minus, dim3((P * P + 255) / 256), dim3(256), 0, st, M, out, P);
    return hipGetLastError();
}

hipError_t cx_reduce_at(hipStream_t st, const double* part, int nwg, int64_t stride, int64_t off, int q, int P,
                        const zd* add, zd* out, const Ctl* ctl) {
    if (q * P <= 0) return hipSuccess;
    hipLaunchKernelGGL(mx::k_cx_reduce, dim3((q * P + 15) / 16), dim3(256), 0, st, part, nwg, stride, off, q, P, add,
                       out, ctl);
    return hipGetLastError();
}

hipError_t cx_reduce(hipStream_t st, const double* part, int nwg, int q, int P, const zd* add, zd* out,
                     const Ctl* ctl) {
    return cx_reduce_at(st, part, nwg, (int64_t)4 * q * P, 0, q, P, add, out, ctl);
}

}  // namespace bgcr
