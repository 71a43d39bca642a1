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

// Two images per block (as the two-image tables kernel): both images'
// strips, IB bytes apart, share the weights and addresses of every (task,
// row); all tasks in one group.  With five or six tasks per wave the second
// image's accumulators wait in its own output (nL >= 4 TPW NT floats, which
// the launcher checks) while the first image's are written, so that the
// compiler keeps both sets in registers without spilling.  Bitwise the
// projections of k_project.
template <int NT, int TPW, int IB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_project2(
    const float *__restrict__ img, int64_t N, ProjShape P, const float2 *__restrict__ dtab,
    float *__restrict__ pmf) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) float lds[];
    const int64_t g0 = 2 * (int64_t)blockIdx.x;
    if (g0 >= N) return;
    const int nimg = N - g0 >= 2 ? 2 : 1;
    const int L = P.L, n = P.n;
    const float *F[2] = {img + g0 * (int64_t)L * L, img + (g0 + nimg - 1) * (int64_t)L * L};
    // the slot table after both images' strips (an opaque offset, as above)
    int off = 2 * (IB / 4);
    asm volatile("" : "+s"(off));
    float acc[2][TPW][4];
    int bad[2];
    project_images2<NT, TPW, 2, 2, IB>(F, nimg, P, dtab, lds, (float4 *)(lds + off),
                                       s4_rows<NT>(L, IB), 0, acc, bad);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr bool kPark = TPW >= 5;
    float *park = pmf + (g0 + 1) * (int64_t)n * L + threadIdx.x;
    if (kPark && nimg == 2) {
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) park[(4 * t + v) * NT] = acc[1][t][v];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (g < nimg) {  // block-uniform
            if (kPark && g == 1) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int t = 0; t < TPW; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[1][t][v] = park[(4 * t + v) * NT];
                // every parked value is back in registers (the loads have
                // returned) before any thread's outputs overwrite the slots
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                __syncthreads();
            }
            float *out = pmf + (g0 + g) * (int64_t)n * L;
            if (!bad[g])
                emit_outputs<TPW>(P, 0, wave, NW, lane, acc[g],
                                  [&](int k, int b, float v) { out[k * L + b] = v; });
            else  // an image with a non-finite value gets an all-NaN projection
                for (int t = threadIdx.x; t < n * L; t += NT) out[t] = __int_as_float(0x7fc00000);
        }
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

template <int NT, int TPW>
static hipError_t launch_project2_t(const float *img, int64_t N, const ProjShape &P,
                                    const float2 *dtab, float *pmf, hipStream_t s) {
    constexpr int IB = kImg2BytesWide;
    const size_t lds = 2 * (size_t)IB + sizeof(float4) * (P.slots + 1);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_project2<NT, TPW, IB>, hipFuncAttributeMaxDynamicSharedMemorySize,
        96 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_project2<NT, TPW, IB>), dim3((unsigned)((N + 1) / 2)), dim3(NT), lds, s,
                       img, N, P, dtab, pmf);
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
    if (s4_supported(g.L)) {  // two images per block where all tasks fit one group of six
        const int64_t table = (int64_t)g.n * g.L;  // room to park the second image's sums
        if (w512 <= 2) return launch_project2_t<512, 2>(img, N, P, t.d32, pmf, s);
        if (w512 <= 4) return launch_project2_t<512, 4>(img, N, P, t.d32, pmf, s);
        if (w512 <= 5 && table >= 4 * 5 * 512)
            return launch_project2_t<512, 5>(img, N, P, t.d32, pmf, s);
        if (w512 <= 6 && table >= 4 * 6 * 512)
            return launch_project2_t<512, 6>(img, N, P, t.d32, pmf, s);
    }
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
