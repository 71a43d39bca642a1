// Line projection of two images at once (the hat-weighted line sum of
// proj_dev.h), for the fused image -> quantile-table kernel.
//
// The work split is that of proj_dev.h: a lane owns one (slot angle, bin)
// item, walks the image rows, and in each row computes the three hat weights
// of its line once for the four angles of the orbit theta, pi/2 - theta,
// pi - theta, pi/2 + theta.  Here the weights also serve a second image:
// per row the lane computes one position, three weights and one LDS address,
// and then does three 16-byte LDS reads and twelve multiply-adds per image.
//
// Strip layout (per image, R strip rows of P positions, 16 bytes each):
// position p = j + 2 of strip row r (image row i = i0 + r) holds the four
// values the four angles read at column j,
//   kind 0: F[i][j]          (theta)
//   kind 1: F[j][i]          (pi/2 - theta: the transposed image)
//   kind 2: F[i][L-1-j]      (pi - theta: the mirrored row)
//   kind 3: F[L-1-j][i]      (pi/2 + theta: the mirrored transposed image)
// each clipped at 0 and masked to the disk, zero for j outside [0, L).  The
// three pixels of a line in one row are positions j2, j2 + 1, j2 + 2
// (j2 = j0 + 2, j0 the first column of the hat), so one address serves all
// twelve products of an image; the second image's strips sit a fixed
// kImg2Bytes further (an immediate offset of the LDS reads).  The sums are
// formed in the order of proj_dev.h (w0 term first), and a row's line
// position depends only on its image row, so the projections are bitwise
// those of the one-image kernels.
#pragma once
#include "proj_dev.h"

namespace sw {

constexpr int kImg2Bytes = 32768;  // strips of the second image: half the 64 KiB region

// Positions per strip row: j = -2 .. L + 2, odd so that consecutive rows
// start in different banks.
__host__ __device__ inline int s4_positions(int L) { return (L + 5) | 1; }
// Strip rows per image that fit kImg2Bytes.
__host__ __device__ inline int s4_rows(int L) {
    const int r = kImg2Bytes / (16 * s4_positions(L));
    return r < L ? r : L;
}

// Staging entries per kind a thread handles per strip (at most R L of them
// per kind, R L <= kImg2Bytes / 16).
template <int NT>
constexpr int s4_groups() {
    return (kImg2Bytes / 16 + NT - 1) / NT;
}

template <int NT, int IMG>
struct Strip4Regs {
    float x[IMG][2][s4_groups<NT>()];
};

// Entry e of a strip of `w` entries per line: line index q = e / w and
// offset o = e - q w (exact in FP32 for these sizes).
__device__ __forceinline__ void s4_entry(int e, int w, float invw, int &q, int &o) {
    q = (int)fmaf((float)e, invw, 0.5f * invw);
    o = e - __mul24(q, w);
}

// Issue the loads of strip rows [i0, i0 + rows) of `nimg` images into
// registers.  Kind 0 walks the strip rows (j fastest), kind 1 the image rows
// j of the transposed strip (r fastest: F[j][i0 .. i0 + rows) is contiguous).
// Every image is read through a buffer resource covering exactly that image.
template <int NT, int IMG>
__device__ __forceinline__ void s4_load(const float *const (&F)[IMG], int nimg, int L, int i0,
                                        int rows, Strip4Regs<NT, IMG> &X) {
    constexpr int G = s4_groups<NT>();
    const int total = rows * L;
    const float invL = 1.f / (float)L, invR = 1.f / (float)rows;
#pragma unroll
    for (int g = 0; g < IMG; ++g) {
        if (g >= nimg) break;  // block-uniform
        const __amdgpu_buffer_rsrc_t img =
            __builtin_amdgcn_make_buffer_rsrc((void *)F[g], (short)0, 4 * L * L, 0x00020000);
#pragma unroll
        for (int it = 0; it < G; ++it) {
            const int e = threadIdx.x + it * NT;
            int r, j, jj, rr;
            s4_entry(e, L, invL, r, j);
            s4_entry(e, rows, invR, jj, rr);
            // entries past the strip read in range and are dropped at the store
            const int o0 = e < total ? __mul24(i0 + r, L) + j : 0;
            const int o1 = e < total ? __mul24(jj, L) + i0 + rr : 0;
            X.x[g][0][it] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(img, 4 * o0, 0, 0));
            X.x[g][1][it] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(img, 4 * o1, 0, 0));
        }
    }
}

// Write the loaded strip: every value to its own position and to the
// mirrored one (kinds 0/2 from the rows, 1/3 from the transposed rows).  A
// non-finite pixel (inside the disk or not) sets bad[g].
template <int NT, int IMG>
__device__ __forceinline__ void s4_store(int nimg, int L, int i0, int rows,
                                         const Strip4Regs<NT, IMG> &X, float *lds, int (&bad)[IMG]) {
    constexpr int G = s4_groups<NT>();
    const int total = rows * L, P4 = 4 * s4_positions(L);
    const int rr2 = (L - 2) * (L - 2);
    const float invL = 1.f / (float)L, invR = 1.f / (float)rows;
#pragma unroll
    for (int g = 0; g < IMG; ++g) {
        if (g >= nimg) break;
        float *S = lds + g * (kImg2Bytes / 4);
        float nf = 0.f;  // becomes NaN once a non-finite value is read
#pragma unroll
        for (int it = 0; it < G; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < total) {
                int r, j, jj, rr;
                s4_entry(e, L, invL, r, j);
                s4_entry(e, rows, invR, jj, rr);
                const float x0 = X.x[g][0][it], x1 = X.x[g][1][it];
                nf = fmaf(x0, 0.f, nf);
                // pixel (i0 + r, j) and pixel (jj, i0 + rr): x^2 + y^2 <= (1 - h)^2
                const int a0 = 2 * j - L + 1, b0 = 2 * (i0 + r) - L + 1;
                const int a1 = 2 * (i0 + rr) - L + 1, b1 = 2 * jj - L + 1;
                const float v0 = __mul24(a0, a0) + __mul24(b0, b0) <= rr2 ? fmaxf(x0, 0.f) : 0.f;
                const float v1 = __mul24(a1, a1) + __mul24(b1, b1) <= rr2 ? fmaxf(x1, 0.f) : 0.f;
                float *row0 = S + __mul24(r, P4), *row1 = S + __mul24(rr, P4);
                row0[4 * (j + 2)] = v0;
                row0[4 * (L + 1 - j) + 2] = v0;
                row1[4 * (jj + 2) + 1] = v1;
                row1[4 * (L + 1 - jj) + 3] = v1;
            }
        }
        if (nf != 0.f) bad[g] = 1;
    }
}

// Accumulate one strip for this wave's tasks and `IMG` images (a missing
// second image reads its zero strips).  Rows pair from even image rows as in
// accumulate_strip.
template <int TPW, int IMG>
__device__ __forceinline__ void s4_accumulate(const LaneTask (&tasks)[TPW], int L,
                                              const float *lds, int i0, int rows,
                                              float (&acc)[IMG][TPW][4], int my_tasks) {
    const float hi3 = (float)L + 2.f;
    const int P16 = 16 * s4_positions(L);
    const int lbase = (int)(uintptr_t)(const __attribute__((address_space(3))) float *)lds;
    int s16;
    asm volatile("v_mov_b32 %0, 16" : "=v"(s16));
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t < my_tasks) {  // wave-uniform
            const LaneTask tk = tasks[t];
            const float k2 = 2.f - 3.f * tk.c;
            float s[IMG][4];
#pragma unroll
            for (int g = 0; g < IMG; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) s[g][v] = acc[g][t][v];
            const int ra = max(tk.rlo - i0, 0), rb = min(tk.rhi - i0 + 1, rows);
            auto row = [&](float um, int rbase) {
                um = __builtin_amdgcn_fmed3f(um, 0.5f, hi3);
                const float fr = __builtin_amdgcn_fractf(um);
                const int j2 = (int)um;
                const float w0 = fmaf(-tk.c, fr, tk.c);
                const float w1 = fmaf(-tk.c, fabsf(tk.k1 - fr), 1.f);
                const float w2 = __builtin_amdgcn_fmed3f(fmaf(tk.c, fr, k2), 0.f, 1.f);
                const int pa = __mul24(j2, s16) + rbase;
#pragma unroll
                for (int g = 0; g < IMG; ++g) {
                    const f32x4v K0 = *(const LdsF4 *)(uintptr_t)(pa + g * kImg2Bytes);
                    const f32x4v K1 = *(const LdsF4 *)(uintptr_t)(pa + g * kImg2Bytes + 16);
                    const f32x4v K2 = *(const LdsF4 *)(uintptr_t)(pa + g * kImg2Bytes + 32);
                    s[g][0] = fmaf(w2, K2.x, fmaf(w1, K1.x, fmaf(w0, K0.x, s[g][0])));
                    s[g][1] = fmaf(w2, K2.y, fmaf(w1, K1.y, fmaf(w0, K0.y, s[g][1])));
                    s[g][2] = fmaf(w2, K2.z, fmaf(w1, K1.z, fmaf(w0, K0.z, s[g][2])));
                    s[g][3] = fmaf(w2, K2.w, fmaf(w1, K1.w, fmaf(w0, K0.w, s[g][3])));
                }
            };
            int rr = ra;
            if (rr < rb && ((i0 + rr) & 1)) {  // odd first row (wave-uniform)
                row(fmaf((float)(i0 + rr - 1), tk.r, tk.A3n), lbase + rr * P16);
                ++rr;
            }
            float fi = (float)(i0 + rr);  // even row index, exact in FP32
            for (; rr + 1 < rb; rr += 2, fi += 2.f) {
                const int rbase = lbase + rr * P16;
                row(fmaf(fi, tk.r, tk.A3), rbase);
                row(fmaf(fi, tk.r, tk.A3n), rbase + P16);
            }
            if (rr < rb) row(fmaf(fi, tk.r, tk.A3), lbase + rr * P16);
#pragma unroll
            for (int g = 0; g < IMG; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[g][t][v] = s[g][v];
        }
    }
}

// Projection of `nimg` <= IMG images for the task group starting at task
// tg0 (tasks tg0 + wave + t NW, t < TPW) into the accumulators; lds holds IMG
// strip buffers of kImg2Bytes.  bad[g] is set when image g holds a
// non-finite value.
template <int NT, int TPW, int IMG>
__device__ void project_images2(const float *const (&F)[IMG], int nimg, const ProjShape &P,
                                const float2 *__restrict__ dtab, float *lds, int tg0,
                                float (&acc)[IMG][TPW][4], int (&bad)[IMG]) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int L = P.L, R = s4_rows(L);
#pragma unroll
    for (int g = 0; g < IMG; ++g) {
        bad[g] = 0;
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[g][t][0] = acc[g][t][1] = acc[g][t][2] = acc[g][t][3] = 0.f;
    }
    const int mine = P.ntasks - tg0 - wave;
    const int my_tasks = mine > 0 ? min(TPW, (mine + NW - 1) / NW) : 0;
    LaneTask tasks[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) tasks[t] = make_task(P, dtab, tg0 + wave + t * NW, lane);
    // the padding positions (and a missing image's strips) stay zero
    __syncthreads();  // the caller may have used the region
    for (int q = threadIdx.x; q < IMG * kImg2Bytes / 16; q += NT)
        *(float4 *)(lds + 4 * q) = make_float4(0.f, 0.f, 0.f, 0.f);
    Strip4Regs<NT, IMG> xs;
    s4_load<NT, IMG>(F, nimg, L, 0, min(R, L), xs);
    for (int i0 = 0; i0 < L; i0 += R) {
        const int rows = min(R, L - i0);
        __syncthreads();
        s4_store<NT, IMG>(nimg, L, i0, rows, xs, lds, bad);
        __syncthreads();
        if (i0 + R < L) s4_load<NT, IMG>(F, nimg, L, i0 + R, min(R, L - i0 - R), xs);
        s4_accumulate<TPW, IMG>(tasks, L, lds, i0, rows, acc, my_tasks);
    }
#pragma unroll
    for (int g = 0; g < IMG; ++g) bad[g] = __syncthreads_or(bad[g]);
}

}  // namespace sw
