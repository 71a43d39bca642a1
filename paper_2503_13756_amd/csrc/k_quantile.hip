// Kernel and launcher of the stand-alone CDF/quantile stage (PMF tables ->
// quantile tables); the device routines are in quant_dev.h.
#include "quant_dev.h"

namespace sw {

template <int NT>
__global__ __launch_bounds__(NT) void k_quantile(const float *__restrict__ pmf, int64_t N,
                                                 QuantShape<NT> S,
                                                 const double2 *__restrict__ d64,
                                                 float *__restrict__ qt, double *__restrict__ aux) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) double ldsd[];  // 16-byte aligned: ds_read_b128 on strips
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const int L = S.L, n = S.n, Q = S.Q;
    double *colS = ldsd;
    float *Ut = (float *)(colS + 2 * n);
    const float *P = pmf + g * (int64_t)n * L;
    quantile_phase<NT>([&](int k, int b) { return P[(int64_t)k * L + b]; }, L, n, Q, S.levels, S.TC,
                       d64, Ut, colS, qt + g * (int64_t)Q * n, aux ? aux + 4 * g : nullptr);
}

template <int NT>
static hipError_t launch_quantiles_t(const float *pmf, int64_t N, Geo g, const AngleTable &t,
                                     float *qt, double *aux, hipStream_t s) {
    QuantShape<NT> S{g.L, g.n, g.Q, g.levels, pick_tc(g.n, g.Q, 68 * 1024)};
    const size_t lds = sizeof(double) * 2 * g.n + sizeof(float) * g.Q * (S.TC + 1);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_quantile<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_quantile<NT>), dim3((unsigned)N), dim3(NT), lds, s, pmf, N, S, t.d64, qt,
                       aux);
    return hipGetLastError();
}

// Small batches take 16 waves per image (columns in parallel); the results
// do not depend on the block size.
hipError_t launch_quantiles(const float *pmf, int64_t N, Geo g, const AngleTable &t, float *qt,
                            double *aux, hipStream_t s, bool small) {
    if (N <= 0) return hipSuccess;
    if (small) return launch_quantiles_t<1024>(pmf, N, g, t, qt, aux, s);
    return launch_quantiles_t<256>(pmf, N, g, t, qt, aux, s);
}

}  // namespace sw
