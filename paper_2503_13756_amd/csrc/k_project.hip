// Kernel and launcher of the stand-alone line projection (images -> PMF
// tables); the device routines are in proj_dev.h.
#include "proj2_dev.h"
#include "proj_dev.h"

namespace sw {

template <int NT, int TPW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kProjMinWaves<NT, TPW>, NT <= 256 ? 2 : 4))) void k_project(const float *__restrict__ img, int64_t N,
                                                ProjShape P, const float2 *__restrict__ dtab,
                                                float *__restrict__ pmf) {
    extern __shared__ __align__(16) float lds[];
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const float *F = img + g * (int64_t)P.L * P.L;
    float *out = pmf + g * (int64_t)P.n * P.L;
    int bad = 0;
    if constexpr (NT == 512) {  // four-kind strips, the slot table after them
        // (an opaque offset: a constant one trips the compiler's LDS cast)
        int off = kStripFloats;
        asm volatile("" : "+s"(off));
        project_image4<NT, TPW>(F, P, dtab, lds, (float4 *)(lds + off), strip4_rows_max(P.L), bad,
                                [&](int k, int b, float v) { out[k * P.L + b] = v; });
    } else
        project_image<NT, TPW>(F, P, dtab, lds, bad,
                               [&](int k, int b, float v) { out[k * P.L + b] = v; });
    if (bad) {
        // an image with a non-finite value gets an all-NaN projection
        __syncthreads();
        for (int t = threadIdx.x; t < P.n * P.L; t += NT) out[t] = __int_as_float(0x7fc00000);
    }
}

// Small batches: one block per (image, task group), so that a single image
// spreads over many compute units.  Every block stages the whole image.
template <int NT>
__global__ __launch_bounds__(NT) void k_project_split(const float *__restrict__ img, int64_t N,
                                                      ProjShape P, const float2 *__restrict__ dtab,
                                                      float *__restrict__ pmf) {
    extern __shared__ __align__(16) float lds[];
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const float *F = img + g * (int64_t)P.L * P.L;
    float *out = pmf + g * (int64_t)P.n * P.L;
    int bad = 0;
    project_group<NT, 1>(F, P, dtab, lds, (int)blockIdx.y * (NT / 64), bad,
                         [&](int k, int b, float v) { out[k * P.L + b] = v; });
    if (bad && blockIdx.y == 0)
        for (int t = threadIdx.x; t < P.n * P.L; t += NT) out[t] = __int_as_float(0x7fc00000);
}

template <int NT, int TPW>
static hipError_t launch_project_t(const float *img, int64_t N, const ProjShape &P,
                                   const float2 *dtab, float *pmf, hipStream_t s) {
    const size_t lds = sizeof(float) * kStripFloats + sizeof(float4) * (P.slots + 1);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_project<NT, TPW>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_project<NT, TPW>), dim3((unsigned)N), dim3(NT), lds, s, img, N, P, dtab,
                       pmf);
    return hipGetLastError();
}

hipError_t launch_project(const float *img, int64_t N, Geo g, const AngleTable &t,
                          const ProjPlan &pp, float *pmf, hipStream_t s, bool split) {
    if (N <= 0) return hipSuccess;
    ProjShape P = proj_shape(g.L, g.n);  // 64 KiB of strips: two blocks per CU
    if (pp.L != g.L || pp.n != g.n || pp.ntasks != P.ntasks) return hipErrorInvalidValue;
    P.perm = pp.perm;
    P.trow = pp.trow;
    if (split) {
        constexpr int NT = 128;
        const int groups = (P.ntasks + NT / 64 - 1) / (NT / 64);
        const size_t lds = sizeof(float) * kStripFloats;
        static const hipError_t attr = hipFuncSetAttribute(
            (const void *)k_project_split<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
            96 * 1024);
        (void)attr;
        hipLaunchKernelGGL((k_project_split<NT>), dim3((unsigned)N, (unsigned)groups), dim3(NT),
                           lds, s, img, N, P, t.d32, pmf);
        return hipGetLastError();
    }
    const int w512 = tasks_per_wave(P.ntasks, 512);
    if (w512 <= 2) return launch_project_t<512, 2>(img, N, P, t.d32, pmf, s);
    if (w512 <= 4) return launch_project_t<512, 4>(img, N, P, t.d32, pmf, s);
    if (w512 <= 5) return launch_project_t<512, 5>(img, N, P, t.d32, pmf, s);
    if (w512 <= 6) return launch_project_t<512, 6>(img, N, P, t.d32, pmf, s);
    if (w512 <= 9) return launch_project_t<512, 9>(img, N, P, t.d32, pmf, s);
    const int w1024 = tasks_per_wave(P.ntasks, 1024);
    if (w1024 <= 9) return launch_project_t<1024, 9>(img, N, P, t.d32, pmf, s);
    if (w1024 <= 12) return launch_project_t<1024, 12>(img, N, P, t.d32, pmf, s);
    // larger task counts run in several task groups
    return launch_project_t<1024, 12>(img, N, P, t.d32, pmf, s);
}

}  // namespace sw
