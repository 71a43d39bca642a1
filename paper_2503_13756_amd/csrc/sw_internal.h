// Internal declarations shared by the kernels and the host runtime of
// libswalign.  Not part of the public ABI (include/swalign.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

constexpr int kMaxL = 256;
constexpr int kMaxN = 512;
constexpr int kMaxQ = 512;
constexpr int kMaxTopK = 8;

// LDS image strips of the projection.  A strip holds R image rows and the
// same R image columns transposed (two "kinds", kKindFloats apart).  A strip
// row is stored as sliding windows: the 16-byte chunk q (floats 4q .. 4q+3
// of the row) holds elements q - kStripPad .. q - kStripPad + 3 of the row
// (zero outside the image), so that the window of four consecutive elements
// starting at element e is the one aligned chunk e + kStripPad, and lanes
// reading neighbouring windows read neighbouring chunks.  Rows hold an odd
// number of chunks, so that consecutive rows start in different banks.
constexpr int kStripPad = 3;
constexpr int kKindFloats = 8192;
constexpr int kStripFloats = 2 * kKindFloats;  // 64 KiB
// chunks per strip row: windows start at elements -3 .. L
__host__ __device__ inline int strip_stride(int L) { return (L + kStripPad + 1) | 1; }
__host__ __device__ inline int strip_row_floats(int L) { return 4 * strip_stride(L); }
__host__ __device__ inline int strip_rows_max(int L) { return kKindFloats / strip_row_floats(L); }
// Rows of the four-kind strips of one image (the persistent mixed tables
// kernel): (L + 5) | 1 positions of 16 bytes per row in the 64 KiB region,
// staged in at most four passes of 512 threads both over the strip's rows of
// ceil(L / 2) column pairs (R <= 4 (512 / H)) and over the H image rows of
// its column runs (R <= 512 / ceil(H / 4)).
__host__ __device__ inline int strip4_rows_max(int L) {
    const int P = (L + 5) | 1, H = (L + 1) >> 1;
    int r = 65536 / (16 * P);
    if (r > L) r = L;
    const int cap = 4 * (512 / H), cap1 = 512 / ((H + 3) / 4);
    if (r > cap) r = cap;
    return r < cap1 ? r : cap1;
}

// Projection work order of one geometry (L, n).  The projection's work
// items are (slot angle, bin) pairs, item = slot * L + bin, in units of 8
// consecutive bins of one slot (the last unit of a slot padded); a task is
// eight units, one item per lane, so that each 8-lane group of a wave reads
// evenly spaced LDS windows.  perm lists the items of task t at
// [64 t, 64 t + 64) (-1 for padding), units grouped so that the lines of a
// task cross nearly the same image rows inside the disk, and trow[t] =
// (first, last) is the range of rows where any of them has a pixel of
// non-zero weight (first > last: none).  Device memory, owned by the context.
__host__ __device__ inline int proj_ntasks(int L, int n) {
    return ((n / 8 + 1) * ((L + 7) / 8) + 7) / 8;
}
struct ProjPlan {
    int L = 0, n = 0, ntasks = 0;
    int *perm = nullptr;   // [ntasks * 64]
    int2 *trow = nullptr;  // [ntasks]
};

struct Geo {
    int L, n, Q, levels;
};

// Device copy of the angle table of one n: d[m] = (cos theta_m, -sin theta_m),
// theta_m = 2 pi m / n, which is also the forward DFT twiddle e^{-2 pi i m/n}.
struct AngleTable {
    int n = 0;
    float2 *d32 = nullptr;   // [n]
    double2 *d64 = nullptr;  // [n]
};

// Result record, identical in layout to sw_result.
struct Result {
    int32_t rot_index;
    float theta_rad;
    float shift_px[2];
    float sw2sq;
    int32_t status;
};
static_assert(sizeof(Result) == 24, "sw_result is 24 bytes");

// ---- launchers (each returns hipGetLastError() after its launches) ----
// split: one block per (image, task group), for batches too small to fill the
// device with one block per image
hipError_t launch_project(const float *img, int64_t N, Geo g, const AngleTable &t,
                          const ProjPlan &pp, float *pmf, hipStream_t s, bool split = false);
hipError_t launch_quantiles(const float *pmf, int64_t N, Geo g, const AngleTable &t, float *qt,
                            double *aux, hipStream_t s, bool small = false);
// Ramp-filtered projections: the stacked [2Q][n] tables of the positive and
// negative parts (per image) from signed [n][L] columns.
hipError_t launch_quantiles_rf(const float *pf, int64_t N, Geo g, const AngleTable &t, float *qt,
                               double *aux, hipStream_t s, bool small = false);
// Ramp filter of C columns of L bins (src may equal dst).  hx: the filter's
// cyclic kernel as a table of 2 LP - 1 floats, hx[t] = h[t - (LP - 1)] for
// |t - (LP - 1)| < L and 0 otherwise, LP = ramp_padded_length(L).
int ramp_padded_length(int L);
hipError_t launch_ramp(const float *src, float *dst, int64_t C, int L, const float *hx,
                       hipStream_t s);
// Fused image -> stacked ramp-filtered tables, for geometries where
// tables_rf_fused_fits() holds; hx as for launch_ramp; per_block as for
// launch_tables.
bool tables_rf_fused_fits(Geo g);
hipError_t launch_tables_rf(const float *img, int64_t N, Geo g, const AngleTable &t,
                            const ProjPlan &pp, const float *hx, float *qt, double *aux,
                            hipStream_t s, int per_block = 2);
// sw2sq of the valid results, and the curve, times f.
hipError_t launch_scale_results(Result *out, int64_t P, float *curve, int n, float f,
                                hipStream_t s);
// Fused image -> quantile table; only for geometries where
// tables_fused_fits() holds (the PMF table must fit in LDS).
bool tables_fused_fits(Geo g);
// per_block: images per block, 2 (weights shared by two images, where the
// geometry allows it) or 1; the results are the same.
hipError_t launch_tables(const float *img, int64_t N, Geo g, const AngleTable &t,
                         const ProjPlan &pp, float *qt, double *aux, hipStream_t s,
                         int per_block = 2);
// Angle spectra of quantile tables: spec[g][w][j] complex, w in [0, n/2],
// j in [0, Q); bf16 != 0 stores bfloat16 pairs instead of float pairs.
hipError_t launch_spectrum(const float *qt, int64_t N, Geo g, const AngleTable &t, void *spec,
                           int bf16, hipStream_t s);
struct PairArgs {
    const float *ref_qt;
    const double *ref_aux;
    const float2 *ref_spec;  // FP32 spectra of the references
    int64_t n_ref;
    const float *img_qt;
    const double *img_aux;
    int64_t n_img;
    const int64_t *pairs;  // nullable
    int64_t n_pairs;
    int mode, bf16, top_k;
    Result *out;
    float *curve;  // nullable
};
hipError_t launch_align_pairs(const PairArgs &a, Geo g, const AngleTable &t, hipStream_t s);
// Max-sliced alignment (rotation only) of every pair: n = 64 or 128.
bool msw_supported(Geo g);
hipError_t launch_align_msw(const PairArgs &a, Geo g, hipStream_t s);
// The same for n = 128 with register-resident angle FFTs; needs a coefficient
// scratch of align128_scratch_bytes() (a.ref_spec must hold the references'
// FP32 spectra).  per_wave: one pair per wave (k_align128w) instead of one
// pair per block (k_align128).
bool align128_supported(Geo g);
size_t align128_scratch_bytes(Geo g, int64_t n_ref);
hipError_t launch_align128(const PairArgs &a, Geo g, const AngleTable &t, float2 *gam,
                           hipStream_t s, bool per_wave = true);

// All reference x image pairs on MFMA (bfloat16 spectra, FP32 accumulate),
// top-k lags per pair, then an FP32 rescore of those lags.
struct MfmaArgs {
    const uint32_t *spec_ref;  // [n_ref][n/2+1][Q] packed bf16 complex
    const uint32_t *spec_img;  // [n_img][n/2+1][Q]
    const float *ref_qt;
    const double *ref_aux;
    int64_t n_ref;
    const float *img_qt;
    const double *img_aux;
    int64_t n_img;
    int mode, top_k;
    int16_t *cand;  // [n_ref * n_img][top_k] scratch
    Result *out;
};
bool mfma_path_supported(Geo g);
hipError_t launch_mfma_all_pairs(const MfmaArgs &a, Geo g, const AngleTable &t, hipStream_t s);

hipError_t launch_fill_synthetic(float *x, int64_t n, hipStream_t s);

}  // namespace sw
