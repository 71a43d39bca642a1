// Line projection of images (the Radon transform of Sec. 2.2, discretised
// as a hat-weighted line sum, i.e. pixel-driven linear interpolation onto the
// detector bins).
//
// Formulation on the GPU: gather, atomic-free.  A lane owns one output bin b
// of one "slot" angle theta in [0, pi/4] and walks the image rows.  In row i
// the line of bin b crosses the row at column u = (b - c0 + s (i - c0))/c + c0
// (c = cos theta >= s = sin theta), and the pixels with non-zero weight are
// the four columns floor(u) - 1 .. floor(u) + 2 (at most three of them are
// non-zero because the pixel spacing along the detector is c >= 1/sqrt 2
// bins).  The four hat weights are shared by four angles of the same orbit
// under the symmetries of the square pixel grid:
//   theta        : F[i][j]            -> bin b
//   pi/2 - theta : F[j][i]            -> bin L-1-b
//   pi - theta   : F[i][L-1-j]        -> bin b
//   pi/2 + theta : F[L-1-j][i]        -> bin b
// and theta + pi is the reversed projection of theta.  So one set of weights
// per (slot, bin, row) feeds up to eight output columns; the angle table is
// built with these symmetries exact.
//
// The image is staged through LDS in strips of R rows together with the same
// R columns transposed, so that all four variants read along LDS rows (lanes
// take consecutive bins, hence near-consecutive columns: conflict-light with
// an odd row stride).  Accumulators live in registers across strips.
#pragma once
#include "sw_internal.h"

namespace sw {

__device__ __forceinline__ bool in_disk(int L, int i, int j) {
    // x^2 + y^2 <= (1 - h)^2 in exact integer form
    const int a = 2 * j - L + 1, b = 2 * i - L + 1, r = L - 2;
    return a * a + b * b <= r * r;
}

struct ProjShape {
    int L, n, S, R, slots, items;
};

__host__ inline ProjShape proj_shape(int L, int n, int lds_floats) {
    ProjShape p;
    p.L = L;
    p.n = n;
    p.S = strip_stride(L);
    p.R = lds_floats / (2 * p.S);
    if (p.R > L) p.R = L;
    p.slots = n / 8 + 1;
    p.items = p.slots * L;
    return p;
}

// Stage image rows [i0, i0 + rows) into Srow[r][S] and image columns
// [i0, i0 + rows) transposed into Tcol[r][S]; masked, clipped, zero padded.
template <int NT>
__device__ void stage_strip(const float *__restrict__ F, const ProjShape &P, int i0, int rows,
                            float *Srow, float *Tcol, int &bad) {
    const int L = P.L, S = P.S;
    for (int r = 0; r < rows; ++r) {
        const int i = i0 + r;
        for (int jj = threadIdx.x; jj < S; jj += NT) {
            const int j = jj - kPadLeft;
            float v = 0.f;
            if (j >= 0 && j < L) {
                const float x = F[(size_t)i * L + j];
                if (!isfinite(x)) bad = 1;
                if (in_disk(L, i, j) && x > 0.f) v = x;
            }
            Srow[r * S + jj] = v;
        }
    }
    // threads as (column block, row): consecutive threads read consecutive
    // image columns of one image row
    const int per = NT / rows;  // rows <= NT is guaranteed by the launcher
    const int r = threadIdx.x % rows;
    const int jb = threadIdx.x / rows;
    if (jb < per) {
        for (int jj = jb; jj < S; jj += per) {
            const int j = jj - kPadLeft;
            float v = 0.f;
            if (j >= 0 && j < L) {
                const int i = i0 + r;
                const float x = F[(size_t)j * L + i];
                if (in_disk(L, j, i) && x > 0.f) v = x;
            }
            Tcol[r * S + jj] = v;
        }
    }
}

// Per-lane constants of one task (slot angle, bin).
struct LaneTask {
    float c, omc, om2c, r, A;
};

__device__ __forceinline__ LaneTask make_task(const ProjShape &P, const float2 *dtab, int item) {
    LaneTask t;
    if (item < P.items) {
        const int slot = item / P.L, b = item - slot * P.L;
        const float2 d = dtab[slot];
        const float c = d.x, s = -d.y;
        const float c0 = 0.5f * (float)(P.L - 1);
        t.c = c;
        t.r = s / c;
        // u(i) = A + i * r
        t.A = ((float)b - c0) / c + c0 - c0 * t.r;
    } else {
        t.c = 1.f;
        t.r = 0.f;
        t.A = -100.f;  // clamps to the zero padding
    }
    t.omc = 1.f - t.c;
    t.om2c = 1.f - 2.f * t.c;
    return t;
}

// Accumulate one LDS strip into the accumulators of this wave's tasks.  Task
// slots are the outer loop (a wave-uniform guard each) and rows the inner,
// unrolled loop, so the LDS reads of consecutive rows are in flight together.
template <int TPW>
__device__ __forceinline__ void accumulate_strip(const ProjShape &P, const float2 *dtab,
                                                 const float *Srow, int i0, int rows, int tg0,
                                                 int wave, int nwaves, int lane,
                                                 float (&acc)[TPW][4], int my_tasks) {
    const int L = P.L, S = P.S;
    const float hi = (float)L + 0.5f;
    // the transposed strip sits R * S floats after the row strip
    const int toff = P.R * S;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t < my_tasks) {  // wave-uniform
            const LaneTask tk = make_task(P, dtab, (tg0 + wave + t * nwaves) * 64 + lane);
            float s0 = acc[t][0], s1 = acc[t][1], s2 = acc[t][2], s3 = acc[t][3];
            const float *row = Srow + kPadLeft;
#pragma unroll 4
            for (int rr = 0; rr < rows; ++rr) {
                float u = fmaf((float)(i0 + rr), tk.r, tk.A);
                u = __builtin_amdgcn_fmed3f(u, -1.5f, hi);
                const float jf = floorf(u);
                const float cf = tk.c * (u - jf);
                const int jA = (int)jf;
                const float w0 = __builtin_amdgcn_fmed3f(tk.omc - cf, 0.f, 1.f);   // column jA - 1
                const float w1 = 1.f - cf;                                          // column jA
                const float w2 = tk.omc + cf;                                       // column jA + 1
                const float w3 = __builtin_amdgcn_fmed3f(tk.om2c + cf, 0.f, 1.f);  // column jA + 2
                const float *a = row + rr * S + jA;
                const float *fa = row + rr * S + (L - 1 - jA);
                const float a0 = a[-1], a1 = a[0], a2 = a[1], a3 = a[2];
                const float b0 = a[toff - 1], b1 = a[toff], b2 = a[toff + 1], b3 = a[toff + 2];
                const float c0 = fa[1], c1 = fa[0], c2 = fa[-1], c3 = fa[-2];
                const float d0 = fa[toff + 1], d1 = fa[toff], d2 = fa[toff - 1], d3 = fa[toff - 2];
                s0 = fmaf(w3, a3, fmaf(w2, a2, fmaf(w1, a1, fmaf(w0, a0, s0))));
                s1 = fmaf(w3, b3, fmaf(w2, b2, fmaf(w1, b1, fmaf(w0, b0, s1))));
                s2 = fmaf(w3, c3, fmaf(w2, c2, fmaf(w1, c1, fmaf(w0, c0, s2))));
                s3 = fmaf(w3, d3, fmaf(w2, d2, fmaf(w1, d1, fmaf(w0, d0, s3))));
            }
            acc[t][0] = s0;
            acc[t][1] = s1;
            acc[t][2] = s2;
            acc[t][3] = s3;
        }
    }
}

// Walk one output value per (task, variant) to its columns, including the
// theta + pi mirror.  Emit(k, b, value) is called for each produced column.
// Tasks of this wave are tg0 + wave + t * nwaves.
template <int TPW, typename Emit>
__device__ __forceinline__ void emit_outputs(const ProjShape &P, int tg0, int wave, int nwaves,
                                             int lane, const float (&acc)[TPW][4], Emit emit) {
    const int L = P.L, n = P.n, q = n / 4, h = n / 2, o = n / 8;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int item = (tg0 + wave + t * nwaves) * 64 + lane;
        if (item >= P.items) continue;
        const int k = item / L, b = item - k * L;
        // variant 0: angle k, bin b
        emit(k, b, acc[t][0]);
        emit(k + h, L - 1 - b, acc[t][0]);
        if (k != o) {  // variant 1: angle n/4 - k, bin L-1-b
            emit(q - k, L - 1 - b, acc[t][1]);
            emit(q - k + h, b, acc[t][1]);
        }
        if (k != 0) {  // variant 2: angle n/2 - k, bin b
            emit(h - k, b, acc[t][2]);
            emit(n - k, L - 1 - b, acc[t][2]);
        }
        if (k != 0 && k != o) {  // variant 3: angle n/4 + k, bin b
            emit(q + k, b, acc[t][3]);
            emit(q + k + h, L - 1 - b, acc[t][3]);
        }
    }
}

// Projection of the tasks [tg0, tg0 + NW * TPW) of one image held in LDS
// strips; results handed to emit.  Returns (in bad_out) whether the image
// holds a non-finite value.
template <int NT, int TPW, typename Emit>
__device__ void project_group(const float *__restrict__ F, const ProjShape &P,
                              const float2 *__restrict__ dtab, float *lds, int tg0, int &bad_out,
                              Emit emit) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[TPW][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = 0.f;
    float *Srow = lds;
    float *Tcol = lds + P.R * P.S;
    const int ntasks = (P.items + 63) / 64;
    const int mine = ntasks - tg0 - wave;
    const int my_tasks = mine > 0 ? min(TPW, (mine + NW - 1) / NW) : 0;
    int bad = 0;
    for (int i0 = 0; i0 < P.L; i0 += P.R) {
        const int rows = min(P.R, P.L - i0);
        __syncthreads();
        stage_strip<NT>(F, P, i0, rows, Srow, Tcol, bad);
        __syncthreads();
        accumulate_strip<TPW>(P, dtab, Srow, i0, rows, tg0, wave, NW, lane, acc, my_tasks);
    }
    bad_out = __syncthreads_or(bad);
    // an image with a non-finite value emits nothing; the caller fills it
    if (!bad_out) emit_outputs<TPW>(P, tg0, wave, NW, lane, acc, emit);
}

// Full projection of one image: as many task groups as needed.  emit must
// not write to the strip buffers (the next group restages them).
template <int NT, int TPW, typename Emit>
__device__ void project_image(const float *__restrict__ F, const ProjShape &P,
                              const float2 *__restrict__ dtab, float *lds, int &bad_out,
                              Emit emit) {
    constexpr int NW = NT / 64;
    const int ntasks = (P.items + 63) / 64;
    bad_out = 0;
    for (int tg0 = 0; tg0 < ntasks; tg0 += NW * TPW) {
        int bad = 0;
        project_group<NT, TPW>(F, P, dtab, lds, tg0, bad, emit);
        bad_out |= bad;
    }
}

// Tasks (64 consecutive work items) per wave for a block of nt threads.
inline int tasks_per_wave(int items, int nt) {
    const int tasks = (items + 63) / 64;
    const int nw = nt / 64;
    return (tasks + nw - 1) / nw;
}

}  // namespace sw
