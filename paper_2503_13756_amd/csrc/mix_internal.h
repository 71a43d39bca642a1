// Declarations of the mixed-geometry persistent launches (k_mixed.hip)
// shared with the host code.
#pragma once
#include "sw_internal.h"

namespace sw {

constexpr int kMaxMix = 64;
// block size and tasks per wave of the persistent tables kernel; launches
// whose every item projects in one task group of five tasks per wave take
// that smaller instance (fewer registers, no spills); the nine-task instance
// (a knob of the autotuner) restages an image for fewer task groups at large
// L (two instead of three at L = n = 256) at three waves per SIMD
constexpr int kMixTablesThreads = 512, kMixTablesTasks = 6, kMixTablesTasksSmall = 5,
              kMixTablesTasksLarge = 9;

// One stack of images of one geometry aligned against one reference.
struct MixItem {
    const float *img;   // [count][L][L]
    float *qt;          // [count][Q][n]
    double *aux;        // [count][4]
    const float *ref_qt;
    const double *ref_aux;
    float2 *ref_spec;   // [n/2+1][Q] FP32, written by the launch
    Result *out;        // [count]
    const float2 *d32;  // angle table of n
    const double2 *d64;
    const int *perm;    // projection work order of (L, n)
    const int2 *trow;
    int64_t first, count;  // work-index range
    int L, n, Q, levels;
    int R;      // projection strip rows (tile)
    int TC;     // quantile column tile
    int fused;  // PMF kept in LDS
    int mode, bf16, top_k;
    float2 *gam;  // n = 128 register-FFT alignment: coefficients [Q/2][130] of the
                  // reference (written by the launch), or null for the LDS-FFT path
    int spec;     // reference item: write the FP32 spectrum of its table to ref_spec
                  // after the tables; image item: its ref_spec is written that way
    int pad;
};
struct MixGroup {
    int64_t total;
    int64_t split;  // work items [0, split) belong to items with gam (listed first)
    int nitems;
    int pad;
    MixItem items[kMaxMix];
};
struct MixLaunch {
    int region_floats, lmax, nmax;
    int tpw;  // tasks per wave of the tables kernel instance
    size_t tables_lds;
    int64_t slot_floats;
    size_t align_lds;
    int align_bpc;  // blocks per compute unit of the per-pair (LDS-FFT) alignment kernel
};
// Launch knobs of the autotuner (0: the default); none changes a result.
struct MixKnobs {
    int tpw = 0;        // kMixTablesTasksSmall, kMixTablesTasks or kMixTablesTasksLarge
    int align_bpc = 0;  // 1 .. 8
};
// Fills the per-item tile fields (R clamped, TC, fused) and the launch sizes;
// knobs, when set, choose the tables kernel instance and the alignment grid.
MixLaunch plan_mixed(MixItem *items, int nitems, MixKnobs knobs = MixKnobs());
// Reference tables and spectra (group d_refs) and image tables (group d_imgs)
// from one work queue, spectra of cached references, alignment (group
// d_imgs).  counters: 4 device words; scratch: grid * slot_floats floats.
// Capturable: no host-side dependence on the contents.
hipError_t launch_mixed(const MixGroup *d_refs, const MixGroup *d_imgs, const MixLaunch &m,
                        unsigned long long *counters, float *scratch, int grid, hipStream_t s);
void prepare_mixed();

}  // namespace sw
