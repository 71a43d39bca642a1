// Ramp filter of the line projections (Sec. 2.2, optional high-pass step:
// each slice multiplied by |xi| before the inverse transform; the
// ramp-filtered distance of Sec. 2.3 and its appendix).  With the filter
// |xi| sampled on the M = 2L point frequency grid of the detector (DC term
// zero) and each column zero-padded to M, the filtered column is the cyclic
// convolution
//   Pf[k][b] = sum_{b'} h[(b - b') mod M] P[k][b'],   b, b' < L,
// i.e. the product of the L x L Toeplitz matrix H[b][b'] = h[b - b'] with the
// columns.  That product runs on the matrix cores in FP32
// (v_mfma_f32_16x16x4_f32): a wave takes 16 columns, keeps their values as B
// fragments (b' = 4 s + lane / 16, column lane % 16), and for each 16-bin
// output tile accumulates the L/4 K-steps with A fragments
// H[16 t + lane % 16][4 s + lane / 16] read from the kernel table in LDS.
// The column is padded to LP = L rounded up to 16 with zeros.
#include "sw_internal.h"

namespace sw {

typedef float f32x4r __attribute__((ext_vector_type(4)));

template <int NS>  // K-steps: LP / 4
__global__ __launch_bounds__(256) void k_ramp(const float *src, float *dst, int64_t C,
                                              int L, const float *__restrict__ hx) {
    constexpr int LP = 4 * NS, NB = LP / 16, HX = 2 * LP - 1;
    __shared__ float hs[HX];  // hs[t] = h[t - (LP - 1)], 0 beyond |t - (LP - 1)| >= L
    for (int i = threadIdx.x; i < HX; i += 256) hs[i] = hx[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t ntiles = (C + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t col = tile * 16 + li;
        const bool cv = col < C;
        const float *P = src + (cv ? col : 0) * (int64_t)L;
        float bf[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int b = 4 * s + lk;
            bf[s] = (cv && b < L) ? P[b] : 0.f;
        }
        float *out = dst + (cv ? col : 0) * (int64_t)L;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            f32x4r acc = {0.f, 0.f, 0.f, 0.f};
            // A[i][k] = h[16 t + i - 4 s - k] at table index 16 t - 4 s + i - k + LP - 1
            const float *ha = hs + 16 * t + li - lk + (LP - 1);
#pragma unroll
            for (int s = 0; s < NS; ++s)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ha[-4 * s], bf[s], acc, 0, 0, 0);
            // this lane holds bins 16 t + 4 (lane / 16) + r of its column
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = 16 * t + 4 * lk + r;
                if (cv && b < L) out[b] = acc[r];
            }
        }
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
