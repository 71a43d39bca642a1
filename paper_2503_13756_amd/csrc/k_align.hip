// Kernels and launchers of the angle spectra and the per-pair alignment;
// the device routines are in align_dev.h.
#include "align_dev.h"

namespace sw {

template <int NT>
__global__ __launch_bounds__(NT) void k_spectrum(const float *__restrict__ qt, int64_t N, Geo g,
                                                 const float2 *__restrict__ tw32, void *spec,
                                                 int bf16) {
    extern __shared__ __align__(16) float2 lds2[];
    const int64_t gi = blockIdx.x;
    if (gi >= N) return;
    const int Wn = g.n / 2 + 1;
    const size_t esz = bf16 ? sizeof(uint32_t) : sizeof(float2);
    spectrum_block<NT>(qt + gi * (int64_t)g.Q * g.n, g.n, g.Q,
                       (char *)spec + (size_t)gi * Wn * g.Q * esz, bf16, tw32, lds2);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_align_pairs(PairArgs a, Geo g,
                                                    const float2 *__restrict__ tw32,
                                                    const double2 *__restrict__ tw64) {
    extern __shared__ __align__(16) float2 lds2[];
    const int n = g.n, Q = g.Q, Wn = n / 2 + 1;
    const int64_t pi = blockIdx.x;
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (pi >= P) return;
    const int64_t r = a.pairs ? a.pairs[2 * pi] : pi / a.n_img;
    const int64_t gi = a.pairs ? a.pairs[2 * pi + 1] : pi % a.n_img;
    const bool in_range = r >= 0 && r < a.n_ref && gi >= 0 && gi < a.n_img;
    PairJob job;
    job.au = a.ref_aux + 4 * (in_range ? r : 0);
    job.av = a.img_aux + 4 * (in_range ? gi : 0);
    job.U = a.ref_qt + (in_range ? r : 0) * (int64_t)Q * n;
    job.V = a.img_qt + (in_range ? gi : 0) * (int64_t)Q * n;
    job.Uh = a.ref_spec + (in_range ? r : 0) * (int64_t)Wn * Q;
    job.res = a.out + pi;
    job.curve = a.curve ? a.curve + pi * n : nullptr;
    int status = 0;
    if (!in_range) status = 3;  // bad pair index
    else if (isnan(job.au[0]) || isnan(job.av[0])) status = 2;
    else if (!(job.au[0] > 0.0) || !(job.av[0] > 0.0)) status = 1;
    job.status = status;
    align_pair_block<NT>(job, g, a.mode, a.bf16, a.top_k, tw32, tw64, lds2);
}

hipError_t launch_spectrum(const float *qt, int64_t N, Geo g, const AngleTable &t, void *spec,
                           int bf16, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    constexpr int NT = 256;
    const size_t lds = sizeof(float2) * (g.n + 2 * kFftElems);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_spectrum<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_spectrum<NT>), dim3((unsigned)N), dim3(NT), lds, s, qt, N, g, t.d32,
                       spec, bf16);
    return hipGetLastError();
}

hipError_t launch_align_pairs(const PairArgs &a, Geo g, const AngleTable &t, hipStream_t s) {
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (P <= 0) return hipSuccess;
    constexpr int NT = 256;
    const int Wn = g.n / 2 + 1;
    const int G = Wn >= NT ? 1 : NT / Wn;
    const size_t lds = sizeof(float2) * (g.n + 2 * kFftElems + Wn * G) + sizeof(double) * g.n;
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_align_pairs<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_align_pairs<NT>), dim3((unsigned)P), dim3(NT), lds, s, a, g, t.d32,
                       t.d64);
    return hipGetLastError();
}

}  // namespace sw
