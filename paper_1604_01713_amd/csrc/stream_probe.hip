// Streaming-rate probe: the memory-system ceiling for a given mix of read and
// written blocks, taken with the row-tile schedule of the block-step sweeps
// (XCD-aware contiguous spans, 16-byte loads and stores, the next tile's
// loads issued before the current one is summed).  It is a measurement aid
// for the roofline of the HBM-bound sweeps, not a step of the method.
#include "bgcr.h"
#include "mfma_sweeps.h"

namespace bgcr {

struct OutPtrs {
    double* p[4];
};

constexpr int STREAM_TILE = 256;  // 16-byte pieces per block and workgroup step

template <int NIN>
__global__ __launch_bounds__(256) void k_stream(int64_t n2, BlockPtrs in, OutPtrs out, int nout) {
    const int t = threadIdx.x;
    const int lw = mx::logical_wg();
    int64_t t0, t1;
    mx::tile_span((n2 + STREAM_TILE - 1) / STREAM_TILE, lw, t0, t1);
    double2 cur[NIN], nxt[NIN];
    auto load = [&](double2 (&v)[NIN], int64_t tile) {
        const int64_t i = tile * STREAM_TILE + t;
#pragma unroll
        for (int b = 0; b < NIN; ++b) v[b] = i < n2 ? ((const double2*)in.p[b])[i] : double2{0.0, 0.0};
    };
    if (t0 < t1) load(nxt, t0);
    for (int64_t k = t0; k < t1; ++k) {
#pragma unroll
        for (int b = 0; b < NIN; ++b) cur[b] = nxt[b];
        if (k + 1 < t1) load(nxt, k + 1);
        double2 s = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NIN; ++b) {
            s.x += cur[b].x;
            s.y += cur[b].y;
        }
        const int64_t i = k * STREAM_TILE + t;
        if (i < n2)
            for (int o = 0; o < nout; ++o) ((double2*)out.p[o])[i] = s;
    }
}

}  // namespace bgcr

using namespace bgcr;

extern "C" int bgcr_stream_probe(const double* const* in, int32_t nin, double* const* out, int32_t nout,
                                 int64_t count, int32_t nwg, void* hip_stream) {
    if (!in || nin < 1 || nin > 16 || nout < 0 || nout > 4 || (nout > 0 && !out) || count < 0 || count % 2 != 0 ||
        nwg < 0)
        return BGCR_ERR_INVALID;
    BlockPtrs ip{};
    OutPtrs op{};
    for (int b = 0; b < nin; ++b) {
        if (!in[b] || ((uintptr_t)in[b] & 15)) return BGCR_ERR_INVALID;
        ip.p[b] = in[b];
    }
    for (int o = 0; o < nout; ++o) {
        if (!out[o] || ((uintptr_t)out[o] & 15)) return BGCR_ERR_INVALID;
        op.p[o] = out[o];
    }
    if (count == 0) return BGCR_OK;
    const int64_t n2 = count / 2;
    const int64_t tiles = (n2 + STREAM_TILE - 1) / STREAM_TILE;
    int64_t g = nwg > 0 ? nwg : 512;
    if (g > tiles) g = tiles;
    hipStream_t st = (hipStream_t)hip_stream;
#define L(N)                                                                                              \
    case N:                                                                                               \
        hipLaunchKernelGGL((k_stream<N>), dim3((unsigned)g), dim3(256), 0, st, n2, ip, op, (int)nout); \
        break;
    switch (nin) {
        L(1) L(2) L(3) L(4) L(5) L(6) L(7) L(8) L(9) L(10) L(11) L(12) L(13) L(14) L(15) L(16)
        default: return BGCR_ERR_INVALID;
    }
#undef L
    return hipGetLastError() == hipSuccess ? BGCR_OK : BGCR_ERR_HIP;
}
