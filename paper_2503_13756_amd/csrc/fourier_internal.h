// Declarations of the Fourier-slice projector (k_fourier.hip) shared with
// the host code.
#pragma once
#include "sw_internal.h"

namespace sw {

// Fourier-slice projector (k_fourier.hip): L even with factors 2 and 3
// (lgL, lgNf: log2 of L and Nf for powers of two, else -1), oversampled
// grid Nf = 2L, H = Nf/2 + 1 stored spectrum columns.  Tables (device,
// context-owned): corr[j] = 1 / phihat((j - L/2) / Nf) for the interpolation
// kernel phi, twf[k] = exp(-2 pi i k / Nf) (k < Nf), twl[k] =
// exp(-2 pi i k / L) (k < L), shift[t] = (-1)^k exp(i pi k / L) with
// k = t for t < L/2 and t - L otherwise.  The scratch holds `slots` regions
// of fourier_slot_bytes; the grid is min(N, slots) persistent blocks.
// targets: per slice point (theta_m, k pi), m < n/2 (n with explicit
// angles), k <= L/2, in that order, five float4 (layout at slice_point in
// k_fourier.hip).
constexpr int kFourierW = 7;    // interpolation kernel width in fine-grid points
constexpr int kFourierPad = 4;  // mirrored spectrum columns kept on each side
struct FourierShape {
    int L, n, Nf, lgNf, lgL, H;
    int mirror;  // 1: slices theta_m = 2 pi m / n, m < n/2, plus their theta + pi
                 // mirrors; 0: n slices at explicit angles (the targets table)
};
struct FourierTabs {
    const float *corr;
    const float2 *twf, *twl, *shift;
    const float4 *targets;
};
// per slot: R [L][Nf/2 + 1] and B [Nf][Nf/2 + 2 kFourierPad] complex
__host__ __device__ inline size_t fourier_slot_elems(int L, int Nf) {
    return (size_t)L * (Nf / 2 + 1) + (size_t)Nf * (Nf / 2 + 2 * kFourierPad);
}
size_t fourier_lds_bytes(int L, int Nf);
size_t fourier_slot_bytes(int L, int Nf);
int fourier_blocks_per_cu(int L, int Nf);  // resident blocks of the projector per CU
hipError_t launch_fourier(const float *img, int64_t N, const FourierShape &S, const FourierTabs &T,
                          void *scratch, int slots, float *pmf, hipStream_t s);

}  // namespace sw
