// Ramp filter of 16 projection columns on the matrix cores (Sec. 2.2,
// optional high-pass step), shared by the stand-alone filter kernel and the
// fused ramp-filtered tables kernel.
//
// With the filter |xi| sampled on the M = 2L point frequency grid of the
// detector (DC term zero) and each column zero-padded to M, the filtered
// column is the cyclic convolution Pf[b] = sum_{b'} h[(b - b') mod M] P[b'],
// b, b' < L: the product of the L x L Toeplitz matrix H[b][b'] = h[b - b']
// with the columns.  A wave takes 16 columns and keeps their values as the B
// fragments of v_mfma_f32_16x16x4_f32 (bin b' = 4 s + lane / 16, column
// lane % 16); every 16-bin output tile accumulates the LP/4 K-steps with A
// fragments H[16 t + lane % 16][4 s + lane / 16] read from the kernel table,
// LP = L rounded up to 16 with zero padding.
#pragma once
#include "sw_internal.h"

namespace sw {

typedef float f32x4r __attribute__((ext_vector_type(4)));

// hs[t] = h[t - (LP - 1)] for |t - (LP - 1)| < L, 0 otherwise (2 LP - 1
// entries, LDS).  ld(j, b) reads bin b of the tile's column j (j < 16, zero
// past the last column), st(j, b, v) writes it; every read happens before
// the first write, so the filter may run in place.
template <int NS, typename Ld, typename St>
__device__ __forceinline__ void ramp_tile(const float *hs, int L, Ld ld, St st) {
    constexpr int LP = 4 * NS, NB = LP / 16;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    float bf[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int b = 4 * s + lk;
        bf[s] = b < L ? ld(li, b) : 0.f;
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        f32x4r acc = {0.f, 0.f, 0.f, 0.f};
        // A[i][k] = h[16 t + i - 4 s - k] at table index 16 t - 4 s + i - k + LP - 1
        const float *ha = hs + 16 * t + li - lk + (LP - 1);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ha[-4 * s], bf[s], acc, 0, 0, 0);
        // this lane holds bins 16 t + 4 (lane / 16) + r of its column
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = 16 * t + 4 * lk + r;
            if (b < L) st(li, b, acc[r]);
        }
    }
}

}  // namespace sw
