// Fused projection + CDF/quantile stage: one block turns one image into its
// quantile table without the projection leaving the chip.  The projection
// accumulates in registers across LDS image strips (proj_dev.h); after the
// last strip the block writes the PMF table into the same LDS region and
// inverts its columns there (quant_dev.h).  Results are identical in form to
// the stand-alone projection followed by the stand-alone quantile stage.
#include "proj_dev.h"
#include "quant_dev.h"

namespace sw {

struct TablesShape {
    ProjShape P;
    int Q, levels, TC;
    int region_floats;  // max(strip buffers, PMF table), a multiple of 2
};

template <int NT, int TPW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kProjMinWaves<NT, TPW>, NT <= 256 ? 2 : 4))) void k_tables(const float *__restrict__ img, int64_t N,
                                               TablesShape T, const float2 *__restrict__ d32,
                                               const double2 *__restrict__ d64,
                                               float *__restrict__ qt, double *__restrict__ aux) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) double ldsd[];  // 16-byte aligned: ds_read_b128 on strips
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const ProjShape &P = T.P;
    const int L = P.L, n = P.n, Q = T.Q;
    float *region = (float *)ldsd;
    double *colS = ldsd + T.region_floats / 2;
    float *Ut = (float *)(colS + 2 * n);
    const float *F = img + g * (int64_t)L * L;
    int bad = 0;
    project_image<NT, TPW>(F, P, d32, region, bad,
                           [&](int k, int b, float v) { region[k * L + b] = v; });
    if (bad)
        for (int t = threadIdx.x; t < n * L; t += NT) region[t] = __int_as_float(0x7fc00000);
    __syncthreads();
    quantile_phase<NT>([&](int k, int b) { return region[k * L + b]; }, L, n, Q, T.levels, T.TC,
                       d64, Ut, colS, qt + g * (int64_t)Q * n, aux ? aux + 4 * g : nullptr);
}

// Bytes of LDS the fused kernel needs for a geometry (0 when it cannot run).
size_t tables_lds_bytes(Geo g, int nt, TablesShape *out) {
    TablesShape T;
    T.P = proj_shape(g.L, g.n);
    T.Q = g.Q;
    T.levels = g.levels;
    // all tasks in one group: the PMF table is written over the strip buffers
    if (tasks_per_wave(T.P.ntasks, nt) > (nt >= 512 ? 9 : 20)) return 0;
    int region = kStripFloats;
    if (region < g.n * g.L) region = g.n * g.L;
    region = (region + 1) & ~1;
    T.region_floats = region;
    const size_t fixed = sizeof(float) * region + sizeof(double) * 2 * g.n;
    // two blocks per CU when the PMF table allows it (160 KiB of LDS per CU)
    const size_t budget2 = 79 * 1024, budget1 = 150 * 1024;
    const size_t budget = fixed + sizeof(float) * g.Q * 9 <= budget2 ? budget2 : budget1;
    if (fixed + sizeof(float) * g.Q * 9 > budget) return 0;
    T.TC = pick_tc(g.n, g.Q, budget - fixed);
    if (out) *out = T;
    return fixed + sizeof(float) * g.Q * (T.TC + 1);
}

bool tables_fused_fits(Geo g) { return tables_lds_bytes(g, 256, nullptr) != 0; }

template <int NT, int TPW>
static hipError_t launch_tables_t(const float *img, int64_t N, const TablesShape &T, size_t lds,
                                  const AngleTable &t, float *qt, double *aux, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_tables<NT, TPW>, hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_tables<NT, TPW>), dim3((unsigned)N), dim3(NT), lds, s, img, N, T, t.d32,
                       t.d64, qt, aux);
    return hipGetLastError();
}

hipError_t launch_tables(const float *img, int64_t N, Geo g, const AngleTable &t,
                         const ProjPlan &pp, float *qt, double *aux, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    TablesShape T;
    size_t lds = tables_lds_bytes(g, 512, &T);
    if (pp.L != g.L || pp.n != g.n || pp.ntasks != proj_ntasks(g.L, g.n))
        return hipErrorInvalidValue;
    T.P.perm = pp.perm;
    T.P.trow = pp.trow;
    if (lds != 0 && lds <= 79 * 1024) {
        const int w = tasks_per_wave(T.P.ntasks, 512);
        if (w <= 2) return launch_tables_t<512, 2>(img, N, T, lds, t, qt, aux, s);
        if (w <= 4) return launch_tables_t<512, 4>(img, N, T, lds, t, qt, aux, s);
        if (w <= 6) return launch_tables_t<512, 6>(img, N, T, lds, t, qt, aux, s);
        if (w <= 9) return launch_tables_t<512, 9>(img, N, T, lds, t, qt, aux, s);
    }
    lds = tables_lds_bytes(g, 256, &T);
    if (lds == 0) return hipErrorInvalidValue;  // caller checks tables_fused_fits first
    T.P.perm = pp.perm;
    T.P.trow = pp.trow;
    const int tpw = tasks_per_wave(T.P.ntasks, 256);
    if (tpw <= 4) return launch_tables_t<256, 4>(img, N, T, lds, t, qt, aux, s);
    if (tpw <= 8) return launch_tables_t<256, 8>(img, N, T, lds, t, qt, aux, s);
    if (tpw <= 12) return launch_tables_t<256, 12>(img, N, T, lds, t, qt, aux, s);
    return launch_tables_t<256, 20>(img, N, T, lds, t, qt, aux, s);
}

}  // namespace sw
