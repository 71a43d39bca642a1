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
    extern __shared__ double ldsd[];
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const int L = S.L, n = S.n, Q = S.Q, TC = S.TC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *C = ldsd + wave * (L + 1);
    float *Ut = (float *)(ldsd + NW * (L + 1));
    const int ldt = TC + 1;
    __shared__ double red[NW][4];
    const float *P = pmf + g * (int64_t)n * L;
    float *U = qt + g * (int64_t)Q * n;
    double E = 0.0, ar = 0.0, ai = 0.0, mass0 = 0.0;
    for (int k0 = 0; k0 < n; k0 += TC) {
        for (int kl = wave; kl < TC; kl += NW) {
            const int k = k0 + kl;
            const float *colp = P + (int64_t)k * L;
            double su, sq;
            const double mass = invert_column([&](int b) { return colp[b]; }, L, Q, S.levels, C,
                                              Ut, ldt, kl, lane, &su, &sq);
            if (k == 0) mass0 = mass;
            su = wave_sum_d(su);
            sq = wave_sum_d(sq);
            const double qbar = su / (double)Q;
            const double2 d = d64[k];
            E += sq;
            ar += qbar * d.x;
            ai += qbar * d.y;
        }
        __syncthreads();
        // rows of the tile to the [Q][n] table
        for (int idx = threadIdx.x; idx < Q * TC; idx += NT) {
            const int j = idx / TC, kl = idx - j * TC;
            U[(int64_t)j * n + k0 + kl] = Ut[j * ldt + kl];
        }
        __syncthreads();
    }
    if (lane == 0) {
        red[wave][0] = E;
        red[wave][1] = ar;
        red[wave][2] = ai;
        red[wave][3] = mass0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && aux) {
        double e = 0, x = 0, y = 0, m0 = 0;
        for (int w = 0; w < NW; ++w) {
            e += red[w][0];
            x += red[w][1];
            y += red[w][2];
        }
        m0 = red[0][3];  // column 0 is handled by wave 0
        double *A = aux + 4 * g;
        A[0] = m0;
        A[1] = e;
        A[2] = x / (double)n;
        A[3] = y / (double)n;
    }
}

hipError_t launch_quantiles(const float *pmf, int64_t N, Geo g, const AngleTable &t, float *qt,
                            double *aux, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    constexpr int NT = 256;
    QuantShape<NT> S{g.L, g.n, g.Q, g.levels, pick_tc(g.n, g.Q, 68 * 1024)};
    const size_t lds = sizeof(double) * (NT / 64) * (g.L + 1) + sizeof(float) * g.Q * (S.TC + 1);
    hipLaunchKernelGGL((k_quantile<NT>), dim3((unsigned)N), dim3(NT), lds, s, pmf, N, S, t.d64, qt,
                       aux);
    return hipGetLastError();
}

}  // namespace sw
