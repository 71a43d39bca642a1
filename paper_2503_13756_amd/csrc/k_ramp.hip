// Stand-alone ramp filter of projection columns (Sec. 2.2, optional
// high-pass step; the ramp-filtered distance of Sec. 2.3): waves take tiles
// of 16 columns (ramp_dev.h).
#include "ramp_dev.h"

namespace sw {

template <int NS>  // K-steps: LP / 4
__global__ __launch_bounds__(256) void k_ramp(const float *src, float *dst, int64_t C, int L,
                                              const float *__restrict__ hx) {
    constexpr int LP = 4 * NS, HX = 2 * LP - 1;
    __shared__ float hs[HX];
    for (int i = threadIdx.x; i < HX; i += 256) hs[i] = hx[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int64_t ntiles = (C + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t c0 = tile * 16;
        ramp_tile<NS>(
            hs, L,
            [&](int j, int b) { return c0 + j < C ? src[(c0 + j) * L + b] : 0.f; },
            [&](int j, int b, float v) {
                if (c0 + j < C) dst[(c0 + j) * L + b] = v;
            });
    }
}

int ramp_padded_length(int L) { return (L + 15) / 16 * 16; }

hipError_t launch_ramp(const float *src, float *dst, int64_t C, int L, const float *hx,
                       hipStream_t s) {
    if (C <= 0) return hipSuccess;
    const int LP = ramp_padded_length(L);
    const int64_t tiles = (C + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    const dim3 grid((unsigned)blocks), block(256);
    switch (LP / 16) {
#define SW_RAMP_CASE(nb)                                                                      \
    case nb:                                                                                  \
        hipLaunchKernelGGL((k_ramp<4 * nb>), grid, block, 0, s, src, dst, C, L, hx);          \
        break;
        SW_RAMP_CASE(1) SW_RAMP_CASE(2) SW_RAMP_CASE(3) SW_RAMP_CASE(4) SW_RAMP_CASE(5)
        SW_RAMP_CASE(6) SW_RAMP_CASE(7) SW_RAMP_CASE(8) SW_RAMP_CASE(9) SW_RAMP_CASE(10)
        SW_RAMP_CASE(11) SW_RAMP_CASE(12) SW_RAMP_CASE(13) SW_RAMP_CASE(14) SW_RAMP_CASE(15)
        SW_RAMP_CASE(16)
#undef SW_RAMP_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Doubles sw2sq of the valid results and the curve: the ramp-filtered
// objective is the sum of the two parts' objectives, each normalised by nQ,
// while the alignment kernels normalise the stacked 2Q-row table by 2nQ.
__global__ void k_scale_results(Result *out, int64_t P, float *curve, int n, float f) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < P && out[i].status == 0) out[i].sw2sq *= f;
    if (curve && i < P * (int64_t)n) curve[i] *= f;
}

hipError_t launch_scale_results(Result *out, int64_t P, float *curve, int n, float f,
                                hipStream_t s) {
    if (P <= 0) return hipSuccess;
    const int64_t m = curve ? P * (int64_t)n : P;
    hipLaunchKernelGGL(k_scale_results, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, out, P,
                       curve, n, f);
    return hipGetLastError();
}

}  // namespace sw
