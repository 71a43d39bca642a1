// Fused projection + CDF/quantile stage: one block turns one image (two, in
// k_tables2) into its quantile table without the projection leaving the
// chip.  The projection accumulates in registers across LDS image strips
// (the four-kind strips of proj2_dev.h for 512-thread blocks, the
// sliding-window strips of proj_dev.h for 256 threads); after the last strip
// the block writes the PMF table into the same LDS region and inverts its
// columns there (quant_dev.h).  Results are bitwise those of the stand-alone
// projection followed by the stand-alone quantile stage.
#include "proj2_dev.h"
#include "proj_dev.h"
#include "quant_dev.h"
#include "ramp_dev.h"

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
    if constexpr (NT == 512)  // four-kind strips; the slot table in the column-sum area
        project_image4<NT, TPW>(F, P, d32, region, (float4 *)colS, strip4_rows_max(L), bad,
                                [&](int k, int b, float v) { region[k * L + b] = v; });
    else
        project_image<NT, TPW>(F, P, d32, region, bad,
                               [&](int k, int b, float v) { region[k * L + b] = v; });
    if (bad)
        for (int t = threadIdx.x; t < n * L; t += NT) region[t] = __int_as_float(0x7fc00000);
    __syncthreads();
    quantile_phase<NT>([&](int k, int b) { return region[k * L + b]; }, L, n, Q, T.levels, T.TC,
                       d64, Ut, colS, qt + g * (int64_t)Q * n, aux ? aux + 4 * g : nullptr);
}

// The same for two images per block (proj2_dev.h): one line position, three
// weights and one LDS address per row serve both images.  The projections
// stay in registers until the strips are done; then each image in turn
// writes its PMF table into the region and inverts it.  Results are bitwise
// those of k_tables.  Only for geometries with one task group of at most six
// tasks per wave.  QM: the column inversion compiled (quant_mode_for(L)).
// With five or six tasks per wave the second image's projections would not
// fit the registers beside the first image's quantile phase: they wait in
// the second image's output table (which the host guarantees holds them,
// kParkFloats) and come back before its own phase.
template <int NT, int TPW>
constexpr int kParkFloats = TPW >= 5 ? TPW * 4 * NT : 0;

template <int NT, int TPW, int QM, int IB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_tables2(
    const float *__restrict__ img, int64_t N, TablesShape T, const float2 *__restrict__ d32,
    const double2 *__restrict__ d64, float *__restrict__ qt, double *__restrict__ aux) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) double ldsd[];
    const int64_t g0 = 2 * (int64_t)blockIdx.x;
    if (g0 >= N) return;
    const int nimg = N - g0 >= 2 ? 2 : 1;
    const ProjShape &P = T.P;
    const int L = P.L, n = P.n, Q = T.Q;
    float *region = (float *)ldsd;
    double *colS = ldsd + T.region_floats / 2;
    float *Ut = (float *)(colS + 2 * n);
    const float *F[2] = {img + g0 * (int64_t)L * L, img + (g0 + nimg - 1) * (int64_t)L * L};
    float acc[2][TPW][4];
    int bad[2];
    // the slot table sits in the column-sum area until the quantile phase
    project_images2<NT, TPW, 2, 2, IB>(F, nimg, P, d32, region, (float4 *)colS,
                                       s4_rows<NT>(L, IB), 0, acc, bad);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *park = qt + (g0 + 1) * (int64_t)Q * n + threadIdx.x;
    if (kParkFloats<NT, TPW> > 0 && nimg == 2) {
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) park[(4 * t + v) * NT] = acc[1][t][v];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (g < nimg) {  // block-uniform
            if (kParkFloats<NT, TPW> > 0 && g == 1) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int t = 0; t < TPW; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[1][t][v] = park[(4 * t + v) * NT];
            }
            __syncthreads();  // strips, or the previous image's PMF, no longer read
                              // (and every parked value is back)
            if (!bad[g])
                emit_outputs<TPW>(P, 0, wave, NW, lane, acc[g],
                                  [&](int k, int b, float v) { region[k * L + b] = v; });
            else
                for (int t = threadIdx.x; t < n * L; t += NT) region[t] = __int_as_float(0x7fc00000);
            __syncthreads();
            quantile_phase<NT, QM>([&](int k, int b) { return region[k * L + b]; }, L, n, Q,
                                   T.levels, T.TC, d64, Ut, colS, qt + (g0 + g) * (int64_t)Q * n,
                               aux ? aux + 4 * (g0 + g) : nullptr);
        }
    }
}

// The ramp-filtered tail of one image whose projections sit in `region`
// (columns L + 4 floats apart): the ramp filter in place on the matrix cores
// (waves take tiles of 16 columns), the positive and the negative part of
// every column inverted into the stacked [2Q][n] table U, and aux (nullable)
// = { smallest part mass (NaN for a NaN value), E and a of the stacked
// table }.  hs: the filter taps in LDS.
template <int NT, int NS>
__device__ void rf_image_tail(const TablesShape &T, float *region, const float *hs,
                              const double2 *__restrict__ d64, float *Ut, double *colS, float *U,
                              double *A) {
    constexpr int NW = NT / 64;
    __shared__ double partA[2][4];
    __shared__ double wmin[NW];
    __shared__ int wnan[NW];
    const ProjShape &P = T.P;
    const int L = P.L, n = P.n, Q = T.Q, ldp = L + 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int tile = wave; tile < (n + 15) / 16; tile += NW) {
        const int c0 = 16 * tile;
        ramp_tile<NS>(
            hs, L, [&](int j, int b) { return c0 + j < n ? region[(c0 + j) * ldp + b] : 0.f; },
            [&](int j, int b, float v) {
                if (c0 + j < n) region[(c0 + j) * ldp + b] = v;
            });
    }
    __syncthreads();
    quantile_phase<NT>([&](int k, int b) { return fmaxf(region[k * ldp + b], 0.f); }, L, n, Q,
                       T.levels, T.TC, d64, Ut, colS, U, partA[0]);
    quantile_phase<NT>([&](int k, int b) { return fmaxf(-region[k * ldp + b], 0.f); }, L, n, Q,
                       T.levels, T.TC, d64, Ut, colS, U + (int64_t)Q * n, partA[1]);
    // smallest part mass over the columns, for the status of the image
    double mn = INFINITY;
    int nan = 0;
    for (int k = wave; k < n; k += NW) {
        double sp = 0.0, sm = 0.0;
        for (int b = lane; b < L; b += 64) {
            const float v = region[k * ldp + b];
            if (v != v) nan = 1;
            sp += (double)fmaxf(v, 0.f);
            sm += (double)fmaxf(-v, 0.f);
        }
        sp = wave_sum_d(sp);
        sm = wave_sum_d(sm);
        mn = fmin(mn, fmin(sp, sm));
    }
    nan = __any(nan);
    if (lane == 0) {
        wmin[wave] = mn;
        wnan[wave] = nan;
    }
    __syncthreads();
    if (threadIdx.x == 0 && A) {
        double m = wmin[0];
        int nb = wnan[0];
        for (int w = 1; w < NW; ++w) {
            m = fmin(m, wmin[w]);
            nb |= wnan[w];
        }
        A[0] = nb ? __longlong_as_double(0x7ff8000000000000LL) : m;
        A[1] = partA[0][1] + partA[1][1];
        A[2] = 0.5 * (partA[0][2] + partA[1][2]);
        A[3] = 0.5 * (partA[0][3] + partA[1][3]);
    }
}

// Fused ramp-filtered tables (ramp-filtered SW of Sec. 2.3): the projection
// as above, written into LDS with a padded column stride, the ramp filter in
// place on the matrix cores (ramp_dev.h; waves take tiles of 16 columns),
// then the positive and the negative part of every column inverted into the
// stacked [2Q][n] table, and aux = { smallest part mass (NaN for a NaN
// value), E and a of the stacked table }.  Same results as sw_project,
// sw_ramp and sw_quantiles_rf in sequence.
template <int NT, int TPW, int NS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kProjMinWaves<NT, TPW>, NT <= 256 ? 2 : 4))) void k_tables_rf(
    const float *__restrict__ img, int64_t N, TablesShape T, const float2 *__restrict__ d32,
    const double2 *__restrict__ d64, const float *__restrict__ hx, float *__restrict__ qt,
    double *__restrict__ aux) {
    constexpr int LP = 4 * NS, HX = 2 * LP - 1;
    extern __shared__ __align__(16) double ldsd[];
    const int64_t g = blockIdx.x;
    if (g >= N) return;
    const ProjShape &P = T.P;
    const int L = P.L, n = P.n, Q = T.Q, ldp = L + 4;
    float *region = (float *)ldsd;
    double *colS = ldsd + T.region_floats / 2;
    float *Ut = (float *)(colS + 2 * n);
    float *hs = Ut + Q * (T.TC + 1);
    const float *F = img + g * (int64_t)L * L;
    int bad = 0;
    // columns ldp = L + 4 floats apart: the filter's 16 columns x 4 bins of
    // one fragment read fall in distinct banks; four-kind strips, the slot
    // table in the column-sum area
    project_image4<NT, TPW>(F, P, d32, region, (float4 *)colS, strip4_rows_max(L), bad,
                            [&](int k, int b, float v) { region[k * ldp + b] = v; });
    if (bad)
        for (int t = threadIdx.x; t < n * ldp; t += NT) region[t] = __int_as_float(0x7fc00000);
    for (int i = threadIdx.x; i < HX; i += NT) hs[i] = hx[i];
    __syncthreads();
    rf_image_tail<NT, NS>(T, region, hs, d64, Ut, colS, qt + g * (int64_t)2 * Q * n,
                          aux ? aux + 4 * g : nullptr);
}

// The same for two images per block (as k_tables2): the two images'
// projections from the same strips and weights (strips kImg2Bytes apart),
// held in registers (the second image's parked in its own output table,
// 2Qn floats, during the first image's tail), then image by image written
// into the region with the padded column stride, filtered and inverted.
// Bitwise the results of k_tables_rf.
template <int NT, int TPW, int NS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_tables2_rf(
    const float *__restrict__ img, int64_t N, TablesShape T, const float2 *__restrict__ d32,
    const double2 *__restrict__ d64, const float *__restrict__ hx, float *__restrict__ qt,
    double *__restrict__ aux) {
    constexpr int NW = NT / 64, LP = 4 * NS, HX = 2 * LP - 1;
    extern __shared__ __align__(16) double ldsd[];
    const int64_t g0 = 2 * (int64_t)blockIdx.x;
    if (g0 >= N) return;
    const int nimg = N - g0 >= 2 ? 2 : 1;
    const ProjShape &P = T.P;
    const int L = P.L, n = P.n, Q = T.Q, ldp = L + 4;
    float *region = (float *)ldsd;
    double *colS = ldsd + T.region_floats / 2;
    float *Ut = (float *)(colS + 2 * n);
    float *hs = Ut + Q * (T.TC + 1);
    const float *F[2] = {img + g0 * (int64_t)L * L, img + (g0 + nimg - 1) * (int64_t)L * L};
    float acc[2][TPW][4];
    int bad[2];
    // the filter taps sit past the quantile tile, out of the strips' way
    for (int i = threadIdx.x; i < HX; i += NT) hs[i] = hx[i];
    project_images2<NT, TPW, 2>(F, nimg, P, d32, region, (float4 *)colS, s4_rows<NT>(L), 0, acc,
                                bad);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *park = qt + (g0 + 1) * (int64_t)2 * Q * n + threadIdx.x;
    if (kParkFloats<NT, TPW> > 0 && nimg == 2) {
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) park[(4 * t + v) * NT] = acc[1][t][v];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (g < nimg) {  // block-uniform
            if (kParkFloats<NT, TPW> > 0 && g == 1) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int t = 0; t < TPW; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[1][t][v] = park[(4 * t + v) * NT];
            }
            __syncthreads();  // strips, or the previous image's columns, no longer read
                              // (and every parked value is back)
            if (!bad[g])
                emit_outputs<TPW>(P, 0, wave, NW, lane, acc[g],
                                  [&](int k, int b, float v) { region[k * ldp + b] = v; });
            else
                for (int t = threadIdx.x; t < n * ldp; t += NT)
                    region[t] = __int_as_float(0x7fc00000);
            __syncthreads();
            rf_image_tail<NT, NS>(T, region, hs, d64, Ut, colS,
                                  qt + (g0 + g) * (int64_t)2 * Q * n,
                                  aux ? aux + 4 * (g0 + g) : nullptr);
        }
    }
}

// Bytes of LDS the fused kernel needs for a geometry (0 when it cannot run),
// with a strip region of at least min_region floats.
size_t tables_lds_bytes(Geo g, int nt, TablesShape *out, int min_region = 0) {
    TablesShape T;
    T.P = proj_shape(g.L, g.n);
    T.Q = g.Q;
    T.levels = g.levels;
    // all tasks in one group: the PMF table is written over the strip buffers
    if (tasks_per_wave(T.P.ntasks, nt) > (nt >= 512 ? 9 : 20)) return 0;
    int region = kStripFloats > min_region ? kStripFloats : min_region;
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

template <int NT, int TPW, int QM, int IB>
static hipError_t launch_tables2_q(const float *img, int64_t N, const TablesShape &T, size_t lds,
                                   const AngleTable &t, float *qt, double *aux, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void *)k_tables2<NT, TPW, QM, IB>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       152 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_tables2<NT, TPW, QM, IB>), dim3((unsigned)((N + 1) / 2)), dim3(NT), lds,
                       s, img, N, T, t.d32, t.d64, qt, aux);
    return hipGetLastError();
}

template <int NT, int TPW, int IB>
static hipError_t launch_tables2_t(const float *img, int64_t N, const TablesShape &T, size_t lds,
                                   const AngleTable &t, float *qt, double *aux, hipStream_t s) {
    if (quant_mode_for(T.P.L) == kQuantHalf)
        return launch_tables2_q<NT, TPW, kQuantHalf, IB>(img, N, T, lds, t, qt, aux, s);
    return launch_tables2_q<NT, TPW, kQuantWave, IB>(img, N, T, lds, t, qt, aux, s);
}

// Launch the two-image kernel for w tasks per wave with image strips IB
// bytes apart (the region holds both) into *e, if an instance fits; false
// (nothing launched) if none does.
template <int IB>
static bool launch_tables2_w(const float *img, int64_t N, Geo g, const TablesShape &T, size_t lds,
                             int w, const AngleTable &t, float *qt, double *aux, hipStream_t s,
                             hipError_t *e) {
    const int64_t table = (int64_t)g.Q * g.n;
    if (w <= 2) *e = launch_tables2_t<512, 2, IB>(img, N, T, lds, t, qt, aux, s);
    else if (w <= 4) *e = launch_tables2_t<512, 4, IB>(img, N, T, lds, t, qt, aux, s);
    else if (w <= 5 && table >= kParkFloats<512, 5>)
        *e = launch_tables2_t<512, 5, IB>(img, N, T, lds, t, qt, aux, s);
    else if (w <= 6 && table >= kParkFloats<512, 6>)
        *e = launch_tables2_t<512, 6, IB>(img, N, T, lds, t, qt, aux, s);
    else
        return false;
    return true;
}

hipError_t launch_tables(const float *img, int64_t N, Geo g, const AngleTable &t,
                         const ProjPlan &pp, float *qt, double *aux, hipStream_t s,
                         int per_block) {
    if (N <= 0) return hipSuccess;
    TablesShape T;
    size_t lds = tables_lds_bytes(g, 512, &T);
    if (pp.L != g.L || pp.n != g.n || pp.ntasks != proj_ntasks(g.L, g.n))
        return hipErrorInvalidValue;
    T.P.perm = pp.perm;
    T.P.trow = pp.trow;
    if (lds != 0 && lds <= 79 * 1024) {
        const int w = tasks_per_wave(T.P.ntasks, 512);
        if (per_block == 2 && s4_supported(g.L)) {
            // two images' strips a little over 32 KiB apart (one more strip
            // row at L = 128) while the block still fits two per CU and the
            // quantile phase keeps its column tile
            TablesShape T2;
            const size_t lds2 = tables_lds_bytes(g, 512, &T2, 2 * kImg2BytesWide / 4);
            hipError_t e = hipSuccess;
            if (lds2 != 0 && lds2 <= 79 * 1024 && T2.TC >= T.TC) {
                T2.P.perm = pp.perm;
                T2.P.trow = pp.trow;
                if (launch_tables2_w<kImg2BytesWide>(img, N, g, T2, lds2, w, t, qt, aux, s, &e))
                    return e;
            }
            if (T.region_floats * 4 >= 2 * kImg2Bytes &&
                launch_tables2_w<kImg2Bytes>(img, N, g, T, lds, w, t, qt, aux, s, &e))
                return e;
        }
        if (w <= 2) return launch_tables_t<512, 2>(img, N, T, lds, t, qt, aux, s);
        if (w <= 4) return launch_tables_t<512, 4>(img, N, T, lds, t, qt, aux, s);
        if (w <= 5) return launch_tables_t<512, 5>(img, N, T, lds, t, qt, aux, s);
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

namespace sw {

// LDS of the fused ramp-filtered kernel: the PMF with stride L + 4, the
// column sums, the quantile tile and the filter table; two 512-thread blocks
// per CU when it fits 79 KiB.  0 when the geometry has no fused form (the
// kernel is instantiated for LP = 64 and 128).
static size_t tables_rf_lds_bytes(Geo g, TablesShape *out) {
    TablesShape T;
    T.P = proj_shape(g.L, g.n);
    T.Q = g.Q;
    T.levels = g.levels;
    const int LP = ramp_padded_length(g.L);
    if (LP != 64 && LP != 128) return 0;
    if (tasks_per_wave(T.P.ntasks, 512) > 6) return 0;
    int region = kStripFloats;
    if (region < g.n * (g.L + 4)) region = g.n * (g.L + 4);
    region = (region + 1) & ~1;
    T.region_floats = region;
    const size_t fixed =
        sizeof(float) * region + sizeof(double) * 2 * g.n + sizeof(float) * (2 * LP - 1);
    const size_t budget = 79 * 1024;
    if (fixed + sizeof(float) * g.Q * 9 > budget) return 0;
    T.TC = pick_tc(g.n, g.Q, budget - fixed);
    if (out) *out = T;
    return fixed + sizeof(float) * g.Q * (T.TC + 1);
}

bool tables_rf_fused_fits(Geo g) { return tables_rf_lds_bytes(g, nullptr) != 0; }

template <int NT, int TPW, int NS>
static hipError_t launch_tables_rf_t(const float *img, int64_t N, const TablesShape &T, size_t lds,
                                     const AngleTable &t, const float *hx, float *qt, double *aux,
                                     hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_tables_rf<NT, TPW, NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
        152 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_tables_rf<NT, TPW, NS>), dim3((unsigned)N), dim3(NT), lds, s, img, N, T,
                       t.d32, t.d64, hx, qt, aux);
    return hipGetLastError();
}

template <int NT, int TPW, int NS>
static hipError_t launch_tables2_rf_t(const float *img, int64_t N, const TablesShape &T,
                                      size_t lds, const AngleTable &t, const float *hx, float *qt,
                                      double *aux, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_tables2_rf<NT, TPW, NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
        152 * 1024);
    (void)attr;
    hipLaunchKernelGGL((k_tables2_rf<NT, TPW, NS>), dim3((unsigned)((N + 1) / 2)), dim3(NT), lds,
                       s, img, N, T, t.d32, t.d64, hx, qt, aux);
    return hipGetLastError();
}

// The two-image ramp-filtered kernel for w tasks per wave into *e, if an
// instance fits (the second image's accumulators park in its 2Qn-float
// table); false (nothing launched) if none does.
template <int NS>
static bool launch_tables2_rf_w(const float *img, int64_t N, Geo g, const TablesShape &T,
                                size_t lds, int w, const AngleTable &t, const float *hx, float *qt,
                                double *aux, hipStream_t s, hipError_t *e) {
    const int64_t table = 2 * (int64_t)g.Q * g.n;
    if (w <= 2) *e = launch_tables2_rf_t<512, 2, NS>(img, N, T, lds, t, hx, qt, aux, s);
    else if (w <= 4) *e = launch_tables2_rf_t<512, 4, NS>(img, N, T, lds, t, hx, qt, aux, s);
    else if (w <= 5 && table >= kParkFloats<512, 5>)
        *e = launch_tables2_rf_t<512, 5, NS>(img, N, T, lds, t, hx, qt, aux, s);
    else if (w <= 6 && table >= kParkFloats<512, 6>)
        *e = launch_tables2_rf_t<512, 6, NS>(img, N, T, lds, t, hx, qt, aux, s);
    else
        return false;
    return true;
}

hipError_t launch_tables_rf(const float *img, int64_t N, Geo g, const AngleTable &t,
                            const ProjPlan &pp, const float *hx, float *qt, double *aux,
                            hipStream_t s, int per_block) {
    if (N <= 0) return hipSuccess;
    TablesShape T;
    const size_t lds = tables_rf_lds_bytes(g, &T);
    if (lds == 0) return hipErrorInvalidValue;  // caller checks tables_rf_fused_fits first
    if (pp.L != g.L || pp.n != g.n || pp.ntasks != proj_ntasks(g.L, g.n))
        return hipErrorInvalidValue;
    T.P.perm = pp.perm;
    T.P.trow = pp.trow;
    const int w = tasks_per_wave(T.P.ntasks, 512);
    const int LP = ramp_padded_length(g.L);
    if (per_block == 2 && s4_supported(g.L) && T.region_floats * 4 >= 2 * kImg2Bytes) {
        hipError_t e = hipSuccess;
        if (LP == 64 ? launch_tables2_rf_w<16>(img, N, g, T, lds, w, t, hx, qt, aux, s, &e)
                     : launch_tables2_rf_w<32>(img, N, g, T, lds, w, t, hx, qt, aux, s, &e))
            return e;
    }
    if (LP == 64) {
        if (w <= 2) return launch_tables_rf_t<512, 2, 16>(img, N, T, lds, t, hx, qt, aux, s);
        if (w <= 4) return launch_tables_rf_t<512, 4, 16>(img, N, T, lds, t, hx, qt, aux, s);
        if (w <= 5) return launch_tables_rf_t<512, 5, 16>(img, N, T, lds, t, hx, qt, aux, s);
        return launch_tables_rf_t<512, 6, 16>(img, N, T, lds, t, hx, qt, aux, s);
    }
    if (w <= 2) return launch_tables_rf_t<512, 2, 32>(img, N, T, lds, t, hx, qt, aux, s);
    if (w <= 4) return launch_tables_rf_t<512, 4, 32>(img, N, T, lds, t, hx, qt, aux, s);
    if (w <= 5) return launch_tables_rf_t<512, 5, 32>(img, N, T, lds, t, hx, qt, aux, s);
    return launch_tables_rf_t<512, 6, 32>(img, N, T, lds, t, hx, qt, aux, s);
}

}  // namespace sw
