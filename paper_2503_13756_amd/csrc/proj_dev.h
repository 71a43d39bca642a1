// Line projection of images (the Radon transform of Sec. 2.2, discretised
// as a hat-weighted line sum, i.e. pixel-driven linear interpolation onto the
// detector bins).
//
// Formulation on the GPU: gather, atomic-free.  A lane owns one output bin b
// of one "slot" angle theta in [0, pi/4] and walks the image rows.  In row i
// the line of bin b crosses the row at column u = (b - c0 + s (i - c0))/c + c0
// (c = cos theta >= s = sin theta), and the pixels with non-zero weight are
// at most three consecutive columns (the hat has half-width 1/c <= sqrt 2
// columns, because the pixel spacing along the detector is c >= 1/sqrt 2
// bins).  The three hat weights are shared by four angles of the same orbit
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
// R columns transposed (layout in sw_internal.h: four shifted copies of each,
// so that every four-pixel window is one aligned 16-byte LDS read), so that
// all four variants read along LDS rows.  Accumulators live in registers
// across strips.  This sliding-window form serves the 256- and 1024-thread
// and split kernels; the 512-thread kernels use the four-kind strips of
// proj2_dev.h (same sums, bitwise), which also reuse the task plan, the line
// weights and the emit step defined here.
#pragma once
#include "sw_internal.h"

namespace sw {

__device__ __forceinline__ bool in_disk(int L, int i, int j) {
    // x^2 + y^2 <= (1 - h)^2 in exact integer form
    const int a = 2 * j - L + 1, b = 2 * i - L + 1, r = L - 2;
    return a * a + b * b <= r * r;
}

struct ProjShape {
    int L, n, S, RS, R, slots, items;  // S chunks, RS floats per strip row
    int ntasks;                        // tasks of 64 lanes (proj_ntasks)
    const int *perm;                   // work order (ProjPlan)
    const int2 *trow;
};

// R: requested strip rows (0: as many as fit).
__host__ inline ProjShape proj_shape(int L, int n, int R = 0) {
    ProjShape p;
    p.L = L;
    p.n = n;
    p.S = strip_stride(L);
    p.RS = strip_row_floats(L);
    const int rmax = strip_rows_max(L) < L ? strip_rows_max(L) : L;
    p.R = (R > 0 && R < rmax) ? R : rmax;
    p.slots = n / 8 + 1;
    p.items = p.slots * L;
    p.ntasks = proj_ntasks(L, n);
    p.perm = nullptr;
    p.trow = nullptr;
    return p;
}

// Masked, clipped pixel (row i, column j) of the image, 0 outside it.
__device__ __forceinline__ float pixel(const float *__restrict__ F, int L, int i, int j) {
    if (j < 0 || j >= L || i < 0 || i >= L) return 0.f;
    const float x = F[(size_t)i * L + j];
    return (in_disk(L, i, j) && x > 0.f) ? x : 0.f;
}

// Value of lane - 1 (0 on lane 0): DPP wave_shr:1.
__device__ __forceinline__ float lane_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// Stage image rows [i0, i0 + rows) and image columns [i0, i0 + rows)
// (transposed) into the strip buffer; masked to the disk, clipped at 0 and
// zero outside the image.  Per kind, the strip rows are walked as one
// sequence of entries (row r, element j) with j = -3 .. S-1; a wave takes 64
// consecutive entries, each lane loads one element, and a lane with j >= 0
// writes chunk j from its own element and those of the three lanes before
// it (DPP shifts), so consecutive waves overlap by three entries.  The image
// is read through a buffer resource covering exactly this image: loads are
// range-checked by the hardware (out-of-range offsets read 0); every element
// outside the image lies outside the disk and is masked.
//
// Staging is split in two: strip_load issues the loads of a strip into
// registers and strip_store writes them to LDS, so that the loads of the
// next strip are in flight while the current one is accumulated.
//
// Entries per kind are rows (S + 3) <= 2048 + 3 rows (rows * 4S fits in
// kKindFloats) and rows <= min(L, 2048 / (L + 4)) <= 43, so at most
// kStripEntries; a wave takes at most strip_groups of them.
constexpr int kStripEntries = kKindFloats / 4 + 3 * 43;
template <int NT>
__host__ __device__ constexpr int strip_groups() {
    return (kStripEntries - kStripPad + (NT / 64) * (64 - kStripPad) - 1) /
           ((NT / 64) * (64 - kStripPad));
}

template <int NT>
struct StripRegs {
    float x[2][strip_groups<NT>()];
};

// Entry f of a strip with W entries per row: strip row r and element j.
__device__ __forceinline__ void strip_entry(int f, int W, float invW, int &r, int &j) {
    r = (int)fmaf((float)f, invW, 0.5f * invW);  // exact for these sizes
    j = f - __mul24(r, W) - kStripPad;
}

template <int NT>
__device__ __forceinline__ void strip_load(const float *__restrict__ F, const ProjShape &P,
                                           int i0, int rows, StripRegs<NT> &R) {
    constexpr int NW = NT / 64, STEP = 64 - kStripPad, G = strip_groups<NT>();
    const int L = P.L, W = P.S + kStripPad, total = rows * W;
    const float invW = 1.f / (float)W;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the lane index is made opaque here, so that the entry arithmetic is
    // redone per strip rather than kept live in registers across strips
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const __amdgpu_buffer_rsrc_t img =
        __builtin_amdgcn_make_buffer_rsrc((void *)F, (short)0, 4 * L * L, 0x00020000);
#pragma unroll
    for (int it = 0; it < G; ++it) {
        const int f0 = wave * STEP + it * NW * STEP;
        if (f0 + kStripPad < total) {  // wave-uniform
            int r, j;
            strip_entry(f0 + lane, W, invW, r, j);
            const int i = i0 + r;
            R.x[0][it] = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(img, 4 * (__mul24(i, L) + j), 0, 0));
            R.x[1][it] = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(img, 4 * (__mul24(j, L) + i), 0, 0));
        }
    }
}

// Writes the strip loaded by strip_load; a non-finite pixel sets `bad`.
template <int NT>
__device__ __forceinline__ void strip_store(const ProjShape &P, int i0, int rows,
                                            const StripRegs<NT> &R, float *lds, int &bad) {
    constexpr int NW = NT / 64, STEP = 64 - kStripPad, G = strip_groups<NT>();
    const int L = P.L, RS = P.RS, W = P.S + kStripPad, total = rows * W;
    const int rr2 = (L - 2) * (L - 2);
    const float invW = 1.f / (float)W;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    float nf = 0.f;  // becomes NaN once a non-finite pixel is read
#pragma unroll
    for (int it = 0; it < G; ++it) {
        const int f0 = wave * STEP + it * NW * STEP;
        if (f0 + kStripPad < total) {  // wave-uniform
            const int f = f0 + lane;
            int r, j;
            strip_entry(f, W, invW, r, j);
            const int a = 2 * j - L + 1, b = 2 * (i0 + r) - L + 1;
            const bool keep = lane >= kStripPad && f < total && j >= 0;
            const bool disk = __mul24(a, a) + __mul24(b, b) <= rr2;
#pragma unroll
            for (int kind = 0; kind < 2; ++kind) {
                const float x = R.x[kind][it];
                nf = fmaf(x, 0.f, nf);
                const float v = disk ? fmaxf(x, 0.f) : 0.f;
                const float v1 = lane_prev(v), v2 = lane_prev(v1), v3 = lane_prev(v2);
                if (keep)
                    *(float4 *)(lds + kind * kKindFloats + __mul24(r, RS) + 4 * j) =
                        make_float4(v3, v2, v1, v);
            }
        }
    }
    if (nf != 0.f) bad = 1;
}

// LDS offset (floats) of the four-element window starting at element e of
// the strip row at rowoff.
__device__ __forceinline__ int window_pos(int e, int rowoff) {
    return rowoff + 4 * (e + kStripPad);
}

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) f32x4v LdsF4;

// Per-lane constants of one task (slot angle, bin): c = cos theta, the
// column step r = tan theta per row, A3 = u(0) - 1/c + 3 (u(i) = A3' + i r is
// the column where the line of bin b crosses row i) and k1 = 2 - 1/c; A3, A3n
// and k1 are rounded once from FP64.
struct LaneTask {
    float c, r, A3, A3n, k1;  // A3n: A3 + r, the offset of the next row
    int rlo, rhi;  // rows the task reads (wave-uniform)
};

// Item of lane `lane` of task `task` in the work order, or -1.
__device__ __forceinline__ int task_item(const ProjShape &P, int task, int lane) {
    return task < P.ntasks ? P.perm[task * 64 + lane] : -1;
}

__device__ __forceinline__ LaneTask make_task(const ProjShape &P, const float2 *dtab, int task,
                                              int lane) {
    LaneTask t;
    const int item = task_item(P, task, lane);
    if (task < P.ntasks) {
        const int2 rr = P.trow[task];
        t.rlo = __builtin_amdgcn_readfirstlane(rr.x);
        t.rhi = __builtin_amdgcn_readfirstlane(rr.y);
    } else {
        t.rlo = 1;
        t.rhi = 0;
    }
    if (item >= 0) {
        const int slot = item / P.L, b = item - slot * P.L;
        const float2 d = dtab[slot];
        const float c = d.x, s = -d.y;
        const double c0 = 0.5 * (double)(P.L - 1);
        t.c = c;
        t.r = s / c;
        const double ic = 1.0 / (double)c;
        const double a3 = ((double)b - c0 - 1.0) * ic + c0 + 3.0 - c0 * (double)t.r;
        t.A3 = (float)a3;
        t.A3n = (float)(a3 + (double)t.r);
        t.k1 = (float)(2.0 - ic);
    } else {
        t.c = 1.f;
        t.r = 0.f;
        t.A3 = -100.f;  // clamps to the zero padding
        t.A3n = -100.f;
        t.k1 = 1.f;
    }
    return t;
}

// One row of one task: the three hat weights of the line at column position
// um (shifted by 3, see below) and the twelve multiply-adds of the four
// variants.  ka / kc are the LDS byte addresses of the windows starting at
// elements -2 and L - 1 of the row; s16 = 16 and m16 = -16 arrive at run
// time, so that each address is one 24-bit multiply-add.
__device__ __forceinline__ void accumulate_row(const LaneTask &tk, float k2, float hi3, float um,
                                               int ka, int kc, int s16, int m16, float &s0,
                                               float &s1, float &s2, float &s3) {
    um = __builtin_amdgcn_fmed3f(um, 0.5f, hi3);
    const float fr = __builtin_amdgcn_fractf(um);  // fractional part, exact
    const int j2 = (int)um;                        // j0 + 2
    const float w0 = fmaf(-tk.c, fr, tk.c);                                // column j0
    const float w1 = fmaf(-tk.c, fabsf(tk.k1 - fr), 1.f);                   // j0 + 1
    const float w2 = __builtin_amdgcn_fmed3f(fmaf(tk.c, fr, k2), 0.f, 1.f);  // j0 + 2
    // window j0 .. j0+3 of the row (and of the transposed column) and the
    // mirrored window L-3-j0 .. L-j0
    const int pa = __mul24(j2, s16) + ka;
    const int pc = __mul24(j2, m16) + kc;
    const f32x4v A = *(const LdsF4 *)(uintptr_t)pa;
    const f32x4v B = *(const LdsF4 *)(uintptr_t)(pa + 4 * kKindFloats);
    const f32x4v C = *(const LdsF4 *)(uintptr_t)pc;
    const f32x4v D = *(const LdsF4 *)(uintptr_t)(pc + 4 * kKindFloats);
    s0 = fmaf(w2, A.z, fmaf(w1, A.y, fmaf(w0, A.x, s0)));
    s1 = fmaf(w2, B.z, fmaf(w1, B.y, fmaf(w0, B.x, s1)));
    s2 = fmaf(w2, C.x, fmaf(w1, C.y, fmaf(w0, C.z, s2)));
    s3 = fmaf(w2, D.x, fmaf(w1, D.y, fmaf(w0, D.z, s3)));
}

// Accumulate one LDS strip into the accumulators of this wave's tasks.  Task
// slots are the outer loop (a wave-uniform guard each) and rows the inner
// loop, two rows per iteration, so the LDS reads of both rows are in flight
// together.  Pairs start at even image rows whatever the strip's first row:
// row 2m sits at 2m r + A3 and row 2m + 1 at 2m r + A3n (the row index steps
// once per pair), so every row's line position, and with it the result, is
// the same for any strip height.
template <int TPW>
__device__ __forceinline__ void accumulate_strip(const ProjShape &P, const LaneTask (&tasks)[TPW],
                                                 const float *lds, int i0, int rows,
                                                 float (&acc)[TPW][4], int my_tasks) {
    const int L = P.L;
    const float hi3 = (float)L + 2.f;
    // LDS byte address of the strip buffer
    const int lbase = (int)(uintptr_t)(const __attribute__((address_space(3))) float *)lds;
    // in vector registers: a multiply-add takes at most one scalar operand
    int s16, m16;
    asm volatile("v_mov_b32 %0, 16\n\tv_mov_b32 %1, -16" : "=v"(s16), "=v"(m16));
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t < my_tasks) {  // wave-uniform
            const LaneTask tk = tasks[t];
            // The hat of half-width 1/c (in columns) around u covers at most
            // three columns, j0 = floor(u - 1/c) + 1 .. j0 + 2.  With
            // f = frac(u - 1/c) their weights are
            //   c (1 - f),   1 - c |2 - 1/c - f|,   max(0, 2 - 3c + c f)
            // (c = cos theta in [1/sqrt 2, 1]).  u - 1/c is carried shifted by
            // 3 and clamped to [0.5, L + 2], so that truncation is the floor
            // and j0 stays in [-2, L]: a line clamped there has its whole hat
            // on columns <= 0 or >= L - 1, outside the disk, and so does the
            // clamped position.
            const float k2 = fmaf(-3.f, tk.c, 2.f);
            float s0 = acc[t][0], s1 = acc[t][1], s2 = acc[t][2], s3 = acc[t][3];
            // only the rows of this strip that the task's lines cross
            const int ra = max(tk.rlo - i0, 0), rb = min(tk.rhi - i0 + 1, rows);
            int rr = ra;
            if (rr < rb && ((i0 + rr) & 1)) {  // odd first row (wave-uniform)
                const int ka = lbase + 4 * window_pos(-2, rr * P.RS);
                const int kc = lbase + 4 * window_pos(L - 1, rr * P.RS);
                accumulate_row(tk, k2, hi3, fmaf((float)(i0 + rr - 1), tk.r, tk.A3n), ka, kc, s16,
                               m16, s0, s1, s2, s3);
                ++rr;
            }
            float fi = (float)(i0 + rr);  // even row index, exact in FP32
            for (; rr + 1 < rb; rr += 2, fi += 2.f) {
                const int ka = lbase + 4 * window_pos(-2, rr * P.RS);
                const int kc = lbase + 4 * window_pos(L - 1, rr * P.RS);
                const int kn = 4 * P.RS;  // next row
                accumulate_row(tk, k2, hi3, fmaf(fi, tk.r, tk.A3), ka, kc, s16, m16, s0, s1, s2,
                               s3);
                accumulate_row(tk, k2, hi3, fmaf(fi, tk.r, tk.A3n), ka + kn, kc + kn, s16, m16,
                               s0, s1, s2, s3);
            }
            if (rr < rb) {
                const int ka = lbase + 4 * window_pos(-2, rr * P.RS);
                const int kc = lbase + 4 * window_pos(L - 1, rr * P.RS);
                accumulate_row(tk, k2, hi3, fmaf(fi, tk.r, tk.A3), ka, kc, s16, m16, s0, s1, s2,
                               s3);
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
        const int item = task_item(P, tg0 + wave + t * nwaves, lane);
        if (item < 0) continue;
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
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float acc[TPW][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = 0.f;
    const int mine = P.ntasks - tg0 - wave;
    const int my_tasks = mine > 0 ? min(TPW, (mine + NW - 1) / NW) : 0;
    // per-lane constants of this wave's tasks, set up once for all strips
    LaneTask tasks[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) tasks[t] = make_task(P, dtab, tg0 + wave + t * NW, lane);
    int bad = 0;
    StripRegs<NT> xs;
    strip_load<NT>(F, P, 0, min(P.R, P.L), xs);
    for (int i0 = 0; i0 < P.L; i0 += P.R) {
        const int rows = min(P.R, P.L - i0);
        __syncthreads();
        strip_store<NT>(P, i0, rows, xs, lds, bad);
        __syncthreads();
        // the next strip's loads fly while this one is accumulated
        if (i0 + P.R < P.L) strip_load<NT>(F, P, i0 + P.R, min(P.R, P.L - i0 - P.R), xs);
        accumulate_strip<TPW>(P, tasks, lds, i0, rows, acc, my_tasks);
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
    bad_out = 0;
    for (int tg0 = 0; tg0 < P.ntasks; tg0 += NW * TPW) {
        int bad = 0;
        project_group<NT, TPW>(F, P, dtab, lds, tg0, bad, emit);
        bad_out |= bad;
    }
}

// Waves per SIMD that a projection kernel of NT threads and TPW tasks per
// wave is compiled for: two 512-thread blocks per compute unit (128 VGPRs)
// while the accumulators and task constants of TPW <= 6 fit.
template <int NT, int TPW>
constexpr int kProjMinWaves = (NT == 512 && TPW <= 6) ? 4 : 1;

// Tasks per wave for a block of nt threads.
inline int tasks_per_wave(int ntasks, int nt) {
    const int nw = nt / 64;
    return (ntasks + nw - 1) / nw;
}

}  // namespace sw
