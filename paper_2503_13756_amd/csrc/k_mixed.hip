// Mixed-geometry persistent kernels: one launch covers many image stacks (or
// serving requests) of different side L, each stack with its own reference.
// Blocks pull work items (one image each) from a device counter; the
// description of the stacks (pointers, geometry, strip-row tile, counts)
// lives in device memory, so a captured graph can be replayed with new
// contents and live counts.  The per-image arithmetic is the same device code
// as the single-geometry kernels (projection, CDF/quantiles, FFT alignment).
#include "align128_dev.h"
#include "align_dev.h"
#include "mix_internal.h"
#include "proj2_dev.h"
#include "proj_dev.h"
#include "quant_dev.h"

namespace sw {

__global__ void k_reset_counters(unsigned long long *c, int n) {
    if (threadIdx.x < n) c[threadIdx.x] = 0ull;
}

// Index of the item whose [first, first + count) range holds work index w.
__device__ __forceinline__ int find_item(const MixGroup *G, int64_t w) {
    int lo = 0, hi = G->nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G->items[mid].first <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NT>
__device__ __forceinline__ int64_t next_work(unsigned long long *counter, int64_t *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(counter, 1ull);
    __syncthreads();
    return *slot;
}

// Images -> quantile tables for every item of two groups: the work queue
// holds the images of G0 (the references) first, then those of G1, so that
// the references, one block each, run beside the first images instead of
// alone on an otherwise idle device.  `scratch` holds one PMF slot of
// slot_floats per block, used by images whose PMF table does not fit in LDS.
template <int NT, int TPW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_tables_mixed(
    const MixGroup *__restrict__ G0, const MixGroup *__restrict__ G1, unsigned long long *counter,
    float *scratch, int64_t slot_floats, int region_floats, int /*lmax*/, int nmax) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) double ldsd[];  // 16-byte aligned: ds_read_b128 on strips
    __shared__ int64_t wslot;
    float *region = (float *)ldsd;
    double *colS = ldsd + region_floats / 2;
    float *Ut = (float *)(colS + 2 * nmax);
    const int64_t total0 = G0->total, total = total0 + G1->total;
    for (;;) {
        int64_t w = next_work<NT>(counter, &wslot);
        if (w >= total) break;
        const MixGroup *G = G0;
        if (w >= total0) {
            G = G1;
            w -= total0;
        }
        const MixItem &it = G->items[find_item(G, w)];
        const int64_t gi = w - it.first;
        ProjShape P;
        P.L = it.L;
        P.n = it.n;
        P.S = strip_stride(it.L);
        P.RS = strip_row_floats(it.L);
        P.R = it.R;  // rows of the four-kind strips (plan_mixed clamps it)
        P.slots = it.n / 8 + 1;
        P.items = P.slots * it.L;
        P.ntasks = proj_ntasks(it.L, it.n);
        P.perm = it.perm;
        P.trow = it.trow;
        const int L = P.L, n = P.n, Q = it.Q;
        float *pmf = it.fused ? region : scratch + (int64_t)blockIdx.x * slot_floats;
        const float *F = it.img + gi * (int64_t)L * L;
        int bad = 0;
        // the slot table sits in the column-sum area until the quantile phase
        project_image4<NT, TPW>(F, P, it.d32, region, (float4 *)colS, P.R, bad,
                                [&](int k, int b, float v) { pmf[k * L + b] = v; });
        if (bad)
            for (int t = threadIdx.x; t < n * L; t += NT) pmf[t] = __int_as_float(0x7fc00000);
        __threadfence_block();
        __syncthreads();
        quantile_phase<NT>([&](int k, int b) { return pmf[k * L + b]; }, L, n, Q, it.levels, it.TC,
                           it.d64, Ut, colS, it.qt + gi * (int64_t)Q * n, it.aux + 4 * gi);
        if (G == G0 && it.spec) {
            // the reference's spectrum, from the table this block just wrote
            __threadfence_block();
            spectrum_block<NT>(it.qt + gi * (int64_t)Q * n, n, Q, it.ref_spec, 0, it.d32,
                               (float2 *)ldsd);
        }
    }
}

// FP32 spectrum of the reference of every item whose reference tables were
// not computed in this launch (cached references): one block per item.
template <int NT>
__global__ __launch_bounds__(NT) void k_refspec_mixed(const MixGroup *__restrict__ G) {
    extern __shared__ __align__(16) float2 lds2[];
    const int i = blockIdx.x;
    if (i >= G->nitems) return;
    const MixItem &it = G->items[i];
    if (it.count <= 0 || it.spec) return;  // spec: written by the tables kernel
    spectrum_block<NT>(it.ref_qt, it.n, it.Q, it.ref_spec, 0, it.d32, lds2);
}

// Register-FFT coefficients of the references of the n = 128 items (after
// k_refspec_mixed): one block per item.
__global__ __launch_bounds__(256) void k_gamma_mixed(const MixGroup *__restrict__ G) {
    const int i = blockIdx.x;
    if (i >= G->nitems) return;
    const MixItem &it = G->items[i];
    if (!it.gam || it.count <= 0) return;
    const int P2 = it.Q / 2;
    for (int idx = threadIdx.x; idx < P2 * (kA128Slots + 2); idx += 256) {
        const int p = idx / (kA128Slots + 2), slot = idx - p * (kA128Slots + 2);
        const float2 c = gamma128_coef(it.ref_spec, it.Q, p, slot);
        if (slot < kA128Slots) it.gam[p * kA128Slots + slot] = c;
        else it.gam[P2 * kA128Slots + 2 * p + (slot - kA128Slots)] = c;
    }
}

// n = 128 items (work items [0, split)): register-FFT alignment, one image
// per wave (align128_wave); each wave pulls its own work items.  The items
// with n = 128 come first and share the angle table of n = 128, which the
// block keeps in LDS.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_align128_mixed(
    const MixGroup *__restrict__ G, unsigned long long *counter) {
    __shared__ float2 tw[128];
    __shared__ __attribute__((aligned(16))) float2 wl[NW * kA128WaveElems];
    const int64_t split = G->split;
    if (split <= 0) return;  // block-uniform
    const float2 *d32 = G->items[0].d32;
    for (int i = threadIdx.x; i < 128; i += 64 * NW) tw[i] = d32[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(counter, 1ull);
        const int64_t w = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane(
                                         (unsigned)(got >> 32)) << 32) |
                                    (unsigned)__builtin_amdgcn_readfirstlane((unsigned)got));
        if (w >= split) break;
        const MixItem &it = G->items[find_item(G, w)];
        const int64_t gi = w - it.first;
        const int P2 = it.Q / 2;
        A128Job job;
        job.U = it.ref_qt;
        job.V = it.qt + gi * (int64_t)it.Q * 128;
        job.au = it.ref_aux;
        job.av = it.aux + 4 * gi;
        job.G = it.gam;
        job.GX = it.gam + (int64_t)P2 * kA128Slots;
        job.d32 = it.d32;
        job.d64 = it.d64;
        job.res = it.out + gi;
        job.curve = nullptr;
        job.Q = it.Q;
        job.L = it.L;
        job.mode = it.mode;
        job.bf16 = it.bf16;
        job.top_k = it.top_k;
        int status = 0;
        if (isnan(job.au[0]) || isnan(job.av[0])) status = 2;
        else if (!(job.au[0] > 0.0) || !(job.av[0] > 0.0)) status = 1;
        job.status = status;
        align128_wave(job, wl + wave * kA128WaveElems, tw);
    }
}

// Other items (work items [split, total)): LDS-FFT alignment of every image
// against the item's reference.
template <int NT>
__global__ __launch_bounds__(NT) void k_align_mixed(const MixGroup *__restrict__ G,
                                                    unsigned long long *counter) {
    extern __shared__ __align__(16) float2 lds2[];
    __shared__ int64_t wslot;
    const int64_t total = G->total, split = G->split;
    for (;;) {
        const int64_t w = split + next_work<NT>(counter, &wslot);
        if (w >= total) break;
        const MixItem &it = G->items[find_item(G, w)];
        const int64_t gi = w - it.first;
        Geo g{it.L, it.n, it.Q, it.levels};
        PairJob job;
        job.U = it.ref_qt;
        job.au = it.ref_aux;
        job.Uh = it.ref_spec;
        job.V = it.qt + gi * (int64_t)it.Q * it.n;
        job.av = it.aux + 4 * gi;
        job.res = it.out + gi;
        job.curve = nullptr;
        int status = 0;
        if (isnan(job.au[0]) || isnan(job.av[0])) status = 2;
        else if (!(job.au[0] > 0.0) || !(job.av[0] > 0.0)) status = 1;
        job.status = status;
        align_pair_block<NT>(job, g, it.mode, it.bf16, it.top_k, it.d32, it.d64, lds2);
    }
}

// LDS and scratch needs of a set of items; fills the per-item tile fields
// (fused, TC) and returns the launch parameters.
MixLaunch plan_mixed(MixItem *items, int nitems, MixKnobs knobs) {
    constexpr int NT = 256;                         // align kernels
    constexpr int NTT = kMixTablesThreads, TPW = kMixTablesTasks;  // tables kernel
    MixLaunch m{};
    m.tpw = kMixTablesTasksSmall;
    int lmax = 8, nmax = 8, region = 0;
    int64_t slot = 0;
    size_t align_lds = 0;
    for (int i = 0; i < nitems; ++i) {
        MixItem &it = items[i];
        int R = it.R > 0 ? it.R : strip4_rows_max(it.L);
        if (R > strip4_rows_max(it.L)) R = strip4_rows_max(it.L);
        if (R > it.L) R = it.L;
        if (R < 1) R = 1;
        if (R > NTT) R = NTT;
        it.R = R;
        const int ntasks = proj_ntasks(it.L, it.n);
        const bool one_group = ntasks <= (NTT / 64) * TPW;
        if (ntasks > (NTT / 64) * kMixTablesTasksSmall) m.tpw = TPW;
        const int strip = kStripFloats;
        const int pmf = it.n * it.L;
        // fused when a single task group and the PMF fits beside nothing else
        it.fused = one_group && pmf <= kStripFloats ? 1 : 0;
        region = max(region, it.fused ? max(strip, pmf) : strip);
        if (!it.fused) slot = max(slot, (int64_t)pmf);
        lmax = max(lmax, it.L);
        nmax = max(nmax, it.n);
        const int Wn = it.n / 2 + 1;
        const int G = Wn >= NT ? 1 : NT / Wn;
        align_lds = max(align_lds, sizeof(float2) * (it.n + 2 * kFftElems + Wn * G) +
                                       sizeof(double) * it.n);
    }
    region = (region + 1) & ~1;
    const size_t fixed = sizeof(float) * region + sizeof(double) * 2 * nmax;
    // two blocks per compute unit whenever the narrowest quantile tile fits
    int qbig = 8;
    for (int i = 0; i < nitems; ++i) qbig = max(qbig, items[i].Q);
    const size_t budget =
        fixed + sizeof(float) * (size_t)qbig * 9 <= 79 * 1024 ? 79 * 1024 : 150 * 1024;
    int qmax = 8;
    for (int i = 0; i < nitems; ++i) {
        MixItem &it = items[i];
        it.TC = pick_tc(it.n, it.Q, budget - fixed);
        qmax = max(qmax, it.Q * (it.TC + 1));
    }
    // tables kernel instance: both handle any item (more task groups with
    // fewer tasks per wave); the knob overrides the smallest-that-fits rule
    if (knobs.tpw == kMixTablesTasksSmall || knobs.tpw == TPW ||
        knobs.tpw == kMixTablesTasksLarge) {
        // the region must still hold the fused PMFs: fused needs one group
        bool ok = true;
        for (int i = 0; i < nitems; ++i)
            if (items[i].fused && proj_ntasks(items[i].L, items[i].n) > (NTT / 64) * knobs.tpw)
                ok = false;
        if (ok) m.tpw = knobs.tpw;
    }
    m.align_bpc = knobs.align_bpc >= 1 && knobs.align_bpc <= 8 ? knobs.align_bpc : 8;
    m.region_floats = region;
    m.lmax = lmax;
    m.nmax = nmax;
    m.tables_lds = fixed + sizeof(float) * qmax;
    m.slot_floats = slot;
    m.align_lds = align_lds;
    return m;
}

void prepare_mixed() {
    constexpr int NT = 256, NTT = kMixTablesThreads, TPW = kMixTablesTasks;
    static const hipError_t a1 = hipFuncSetAttribute(
        (const void *)k_tables_mixed<NTT, TPW>, hipFuncAttributeMaxDynamicSharedMemorySize,
        150 * 1024);
    static const hipError_t a0 = hipFuncSetAttribute(
        (const void *)k_tables_mixed<NTT, kMixTablesTasksSmall>,
        hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)a0;
    static const hipError_t a4 = hipFuncSetAttribute(
        (const void *)k_tables_mixed<NTT, kMixTablesTasksLarge>,
        hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)a4;
    static const hipError_t a2 = hipFuncSetAttribute(
        (const void *)k_refspec_mixed<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    static const hipError_t a3 = hipFuncSetAttribute(
        (const void *)k_align_mixed<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)a1;
    (void)a2;
    (void)a3;
}

// Every kernel of the sequence reads its item and work counts from the
// descriptors in device memory, so the sequence can be captured once and
// replayed with new descriptor contents.
hipError_t launch_mixed(const MixGroup *d_refs, const MixGroup *d_imgs, const MixLaunch &m,
                        unsigned long long *counters, float *scratch, int grid, hipStream_t s) {
    constexpr int NT = 256, NTT = kMixTablesThreads, TPW = kMixTablesTasks;
    prepare_mixed();
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters, 4);
    if (m.tpw == kMixTablesTasksSmall)
        hipLaunchKernelGGL((k_tables_mixed<NTT, kMixTablesTasksSmall>), dim3((unsigned)grid),
                           dim3(NTT), m.tables_lds, s, d_refs, d_imgs, counters + 0, scratch,
                           m.slot_floats, m.region_floats, m.lmax, m.nmax);
    else if (m.tpw == kMixTablesTasksLarge)
        hipLaunchKernelGGL((k_tables_mixed<NTT, kMixTablesTasksLarge>), dim3((unsigned)grid),
                           dim3(NTT), m.tables_lds, s, d_refs, d_imgs, counters + 0, scratch,
                           m.slot_floats, m.region_floats, m.lmax, m.nmax);
    else
        hipLaunchKernelGGL((k_tables_mixed<NTT, TPW>), dim3((unsigned)grid), dim3(NTT),
                           m.tables_lds, s, d_refs, d_imgs, counters + 0, scratch,
                           m.slot_floats, m.region_floats, m.lmax, m.nmax);
    hipLaunchKernelGGL((k_refspec_mixed<NT>), dim3((unsigned)kMaxMix), dim3(NT),
                       sizeof(float2) * (kMaxN + 2 * kFftElems), s, d_imgs);
    hipLaunchKernelGGL(k_gamma_mixed, dim3((unsigned)kMaxMix), dim3(256), 0, s, d_imgs);
    // four 37 KiB blocks of four waves of the register-FFT kernel per compute unit
    hipLaunchKernelGGL((k_align128_mixed<4>), dim3((unsigned)(2 * grid)), dim3(256), 0, s, d_imgs,
                       counters + 3);
    // small LDS tiles: several blocks of the LDS-FFT kernel per compute unit
    // (grid = 2 blocks per compute unit; align_bpc per compute unit here)
    hipLaunchKernelGGL((k_align_mixed<NT>), dim3((unsigned)(m.align_bpc * (grid / 2))), dim3(NT),
                       m.align_lds, s, d_imgs, counters + 2);
    return hipGetLastError();
}

// Deterministic synthetic images for timing (autotuner): a hash of the
// element index mapped to [0, 1).
__global__ void k_fill_synthetic(float *x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        x[i] = (float)(h >> 8) * (1.0f / 16777216.0f);
    }
}

hipError_t launch_fill_synthetic(float *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_synthetic, dim3(1024), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

}  // namespace sw
