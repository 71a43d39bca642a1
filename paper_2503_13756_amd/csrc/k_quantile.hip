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

// Ramp-filtered projections (signed) -> stacked quantile tables: rows 0..Q-1
// invert the positive part max(Pf, 0) of every column, rows Q..2Q-1 the
// negative part max(-Pf, 0), each normalised on its own (ramp-filtered SW of
// Sec. 2.3 and its appendix).  aux = { smallest part mass over the columns
// (NaN if a value is NaN), E of the stacked table, a of the stacked table =
// the mean of the two parts' moments }.
template <int NT>
__global__ __launch_bounds__(NT) void k_quantile_rf(const float *__restrict__ pf, int64_t N,
                                                    QuantShape<NT> S,
                                                    const double2 *__restrict__ d64,
                                                    float *__restrict__ qt,
                                                    double *__restrict__ aux) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) double ldsd[];
    __shared__ double partA[2][4];
    __shared__ double wmin[NW];
    __shared__ int wnan[NW];
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const int L = S.L, n = S.n, Q = S.Q;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *colS = ldsd;
    float *Ut = (float *)(colS + 2 * n);
    const float *P = pf + g * (int64_t)n * L;
    float *U = qt + g * (int64_t)2 * Q * n;
    quantile_phase<NT>([&](int k, int b) { return fmaxf(P[(int64_t)k * L + b], 0.f); }, L, n, Q,
                       S.levels, S.TC, d64, Ut, colS, U, partA[0]);
    quantile_phase<NT>([&](int k, int b) { return fmaxf(-P[(int64_t)k * L + b], 0.f); }, L, n,
                       Q, S.levels, S.TC, d64, Ut, colS, U + (int64_t)Q * n, partA[1]);
    // smallest part mass over the columns, for the status of the image
    double mn = INFINITY;
    int bad = 0;
    for (int k = wave; k < n; k += NW) {
        double sp = 0.0, sm = 0.0;
        for (int b = lane; b < L; b += 64) {
            const float v = P[(int64_t)k * L + b];
            if (v != v) bad = 1;
            sp += (double)fmaxf(v, 0.f);
            sm += (double)fmaxf(-v, 0.f);
        }
        sp = wave_sum_d(sp);
        sm = wave_sum_d(sm);
        mn = fmin(mn, fmin(sp, sm));
    }
    bad = __any(bad);
    if (lane == 0) {
        wmin[wave] = mn;
        wnan[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0 && aux) {
        double m = wmin[0];
        int nb = wnan[0];
        for (int w = 1; w < NW; ++w) {
            m = fmin(m, wmin[w]);
            nb |= wnan[w];
        }
        double *A = aux + 4 * g;
        A[0] = nb ? __longlong_as_double(0x7ff8000000000000LL) : m;
        A[1] = partA[0][1] + partA[1][1];
        A[2] = 0.5 * (partA[0][2] + partA[1][2]);
        A[3] = 0.5 * (partA[0][3] + partA[1][3]);
    }
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


template <int NT>
static hipError_t launch_quantiles_rf_t(const float *pf, int64_t N, Geo g, const AngleTable &t,
                                        float *qt, double *aux, hipStream_t s) {
    QuantShape<NT> S{g.L, g.n, g.Q, g.levels, pick_tc(g.n, g.Q, 68 * 1024)};
    const size_t lds = sizeof(double) * 2 * g.n + sizeof(float) * g.Q * (S.TC + 1);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_quantile_rf<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_quantile_rf<NT>), dim3((unsigned)N), dim3(NT), lds, s, pf, N, S, t.d64,
                       qt, aux);
    return hipGetLastError();
}

hipError_t launch_quantiles_rf(const float *pf, int64_t N, Geo g, const AngleTable &t, float *qt,
                               double *aux, hipStream_t s, bool small) {
    if (N <= 0) return hipSuccess;
    if (small) return launch_quantiles_rf_t<1024>(pf, N, g, t, qt, aux, s);
    return launch_quantiles_rf_t<256>(pf, N, g, t, qt, aux, s);
}

}  // namespace sw
