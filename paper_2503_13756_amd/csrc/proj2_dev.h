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
// values the four angles read at column j, in the order
//   F[i][j]          (theta)
//   F[i][L-1-j]      (pi - theta: the mirrored row)
//   F[j][i]          (pi/2 - theta: the transposed image)
//   F[L-1-j][i]      (pi/2 + theta: the mirrored transposed image)
// each clipped at 0 and masked to the disk, zero for j outside [0, L).  The
// three pixels of a line in one row are positions j2, j2 + 1, j2 + 2
// (j2 = j0 + 2, j0 the first column of the hat), so one address serves all
// twelve products of an image; the second image's strips sit a fixed
// kImg2Bytes further (an immediate offset of the LDS reads).  The sums are
// formed in the order of proj_dev.h (w0 term first), and a row's line
// position depends only on its image row, so the projections are bitwise
// those of the one-image kernels.
//
// Staging goes by mirrored pairs: a pixel and its mirror image in the row
// (F[i][j], F[i][L-1-j]) fill the first half of positions j + 2 and
// L + 1 - j (in swapped order), and the column pair (F[j][i], F[L-1-j][i])
// the second half of the same positions, so each loaded pair is two 8-byte
// LDS writes; both pixels of a pair lie at the same distance from the centre,
// so one disk test serves both.
#pragma once
#include "proj_dev.h"

namespace sw {

// strips of the second image: half the 64 KiB region, or a little more where
// the block's LDS allows it (k_tables2's IB)
constexpr int kImg2Bytes = 32768, kImg2BytesWide = 34816;

// Positions per strip row: j = -2 .. L + 2, odd so that consecutive rows
// start in different banks.
__host__ __device__ inline int s4_positions(int L) { return (L + 5) | 1; }
// Column pairs per row: j < ceil(L / 2) (an odd L's middle column pairs with
// itself).
__host__ __device__ inline int s4_pairs(int L) { return (L + 1) >> 1; }
// Strip rows per image: as many as fit `bytes`, at most KP times the rows one
// pass of NT threads covers (so that KP passes stage the row pairs of any
// strip), and at most NT / ceil(H / KP) (so that KP passes of NT / R image
// rows stage the H column pairs); any smaller R satisfies both.
template <int NT = 512, int KP = 2>
__host__ __device__ inline int s4_rows(int L, int bytes = kImg2Bytes) {
    int r = bytes / (16 * s4_positions(L));
    if (r > L) r = L;
    const int H = s4_pairs(L);
    const int cap = KP * (NT / H), cap1 = NT / ((H + KP - 1) / KP);
    if (r > cap) r = cap;
    return r < cap1 ? r : cap1;
}
// Whether the staging covers L with 512-thread blocks.
__host__ __device__ inline bool s4_supported(int L) { return L >= 2 && s4_pairs(L) <= 512; }
// The one-image form: four passes, strips in the whole 64 KiB region
// (strip4_rows_max(L) = s4_rows<512, 4>(L, 65536)).
constexpr int kImg1Passes = 4;

// Loaded strip entries of a thread: [image][row pairs | column pairs][pass]
// [pixel, mirrored pixel].
template <int IMG, int KP>
struct Strip4Regs {
    float x[IMG][2][KP][2];
};

// Quotient and remainder of e by w through a multiply-high with
// mg = floor((2^32 - 1) / w) + 1: exact while e w < 2^32 (e < 512, w <= 1024
// here).  mg is uniform, so each division is one VALU operation with a scalar
// operand.  For w = 1 the multiplier (2^32) does not fit: mg = 0 there and the
// quotient is e itself.
__device__ __forceinline__ void s4_divmod(int e, int w, unsigned mg, int &q, int &o) {
    q = (int)__umulhi((unsigned)e, mg) + (w == 1 ? e : 0);
    o = e - __mul24(q, w);
}

// Per-block constants of the staging: pairs per row H, strip rows R (at most
// s4_rows for the pass count), and the rows a pass covers for each entry kind
// (rp strip rows of pairs, jp image rows of column runs).
struct S4Geo {
    int H, R, rp, jp;
    unsigned mH, mR;  // multipliers of s4_divmod for H and R
};
template <int NT>
__device__ __forceinline__ S4Geo s4_geo(int L, int R) {
    S4Geo G;
    G.H = s4_pairs(L);
    G.R = R;
    G.rp = NT / G.H;
    G.jp = NT / G.R;
    G.mH = G.H > 1 ? 0xffffffffu / (unsigned)G.H + 1u : 0u;
    G.mR = G.R > 1 ? 0xffffffffu / (unsigned)G.R + 1u : 0u;
    // uniform: keep them in scalar registers
    G.rp = __builtin_amdgcn_readfirstlane(G.rp);
    G.jp = __builtin_amdgcn_readfirstlane(G.jp);
    G.mH = __builtin_amdgcn_readfirstlane(G.mH);
    G.mR = __builtin_amdgcn_readfirstlane(G.mR);
    return G;
}

// The thread's entries: row pairs (j0, L-1-j0) of strip rows r0 + k rp, and
// column runs: column i0 + rr0 of image rows jj0 + k jp and L-1-(jj0 + k jp),
// k < KP.  Threads past a full pass (r0 >= rp, jj0 >= jp) have no entries.
struct S4Map {
    int j0, r0, rr0, jj0;
};
// Recomputed at each use (an opaque copy of the thread index keeps the
// compiler from holding the map, loop-invariant, across the accumulation).
__device__ __forceinline__ S4Map s4_map(const S4Geo &G) {
    S4Map m;
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    s4_divmod(t, G.H, G.mH, m.r0, m.j0);
    s4_divmod(t, G.R, G.mR, m.jj0, m.rr0);
    return m;
}

// Issue the loads of strip rows [i0, i0 + R) of `nimg` images into
// registers.  Row pairs read along the strip rows, column runs along image
// rows (F[jj][i0 .. i0 + R) is contiguous), both coalesced.  Every image is
// read through a buffer resource covering exactly that image: entries past
// the image (or with a negative offset) load 0 under the hardware range
// check, entries past the strip load in range; the store drops both.
template <int NT, int IMG, int KP>
__device__ __forceinline__ void s4_load(const float *const (&F)[IMG], int nimg, int L, int i0,
                                        const S4Geo &G, Strip4Regs<IMG, KP> &X) {
    const S4Map m = s4_map(G);
    int o[2][KP][2];
    const int dm = L - 1 - 2 * m.j0;           // F[i][L-1-j0] - F[i][j0]
    const int c = i0 + m.rr0, cm = (L - 1) * L + 2 * c;  // F[L-1-jj][c] = cm - F[jj][c]
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        o[0][k][0] = __mul24(i0 + m.r0 + k * G.rp, L) + m.j0;
        o[0][k][1] = o[0][k][0] + dm;
        o[1][k][0] = __mul24(m.jj0 + k * G.jp, L) + c;
        o[1][k][1] = cm - o[1][k][0];
    }
#pragma unroll
    for (int g = 0; g < IMG; ++g) {
        if (g >= nimg) break;  // block-uniform
        const __amdgpu_buffer_rsrc_t img =
            __builtin_amdgcn_make_buffer_rsrc((void *)F[g], (short)0, 4 * L * L, 0x00020000);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < KP; ++k)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    X.x[g][h][k][v] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(img, 4 * o[h][k][v], 0, 0));
    }
}

// Write the loaded strip (rows [i0, i0 + rows)): clip at 0, mask to the disk
// x^2 + y^2 <= (1 - h)^2, and put each pair into its two positions.  A
// non-finite pixel (inside the disk or not) sets bad[g]; every pixel of the
// image passes through the row pairs once.
template <int NT, int IMG, int KP, int IB = kImg2Bytes>
__device__ __forceinline__ void s4_store(int nimg, int L, int i0, int rows, const S4Geo &G,
                                         const Strip4Regs<IMG, KP> &X, float *lds,
                                         int (&bad)[IMG]) {
    typedef float f32x2v __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) f32x2v LdsF2;
    const S4Map m = s4_map(G);
    const int P16 = 16 * s4_positions(L), rr2 = (L - 2) * (L - 2);
    const int lb = (int)(uintptr_t)(const __attribute__((address_space(3))) float *)lds;
    float nf[IMG];
#pragma unroll
    for (int g = 0; g < IMG; ++g) nf[g] = 0.f;  // becomes NaN once a non-finite value is read
    {  // row pairs: positions j0 + 2 and L + 1 - j0 of strip row r0 + k rp, bytes 0..7
        const int a = 2 * m.j0 - L + 1, a2 = __mul24(a, a);
        const int p0 = lb + __mul24(m.r0, P16) + 16 * (m.j0 + 2);
        const int p1 = p0 + 16 * (L - 1 - 2 * m.j0);
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int r = m.r0 + k * G.rp;
            if (m.r0 < G.rp && r < rows) {
                const int b = 2 * (i0 + r) - L + 1;
                const bool in = __mul24(b, b) + a2 <= rr2;
                const int dk = k * G.rp * P16;
#pragma unroll
                for (int g = 0; g < IMG; ++g) {
                    if (g >= nimg) break;
                    const float x = X.x[g][0][k][0], y = X.x[g][0][k][1];
                    nf[g] = fmaf(y, 0.f, fmaf(x, 0.f, nf[g]));
                    const float u = in ? fmaxf(x, 0.f) : 0.f, v = in ? fmaxf(y, 0.f) : 0.f;
                    *(LdsF2 *)(uintptr_t)(p0 + dk + g * IB) = f32x2v{u, v};
                    *(LdsF2 *)(uintptr_t)(p1 + dk + g * IB) = f32x2v{v, u};
                }
            }
        }
    }
    {  // column runs: positions jj + 2 and L + 1 - jj of strip row rr0, bytes 8..15
        const int a = 2 * (i0 + m.rr0) - L + 1, a2 = __mul24(a, a);
        const int p0 = lb + __mul24(m.rr0, P16) + 16 * (m.jj0 + 2) + 8;
        const int p1 = lb + __mul24(m.rr0, P16) + 16 * (L + 1 - m.jj0) + 8;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int jj = m.jj0 + k * G.jp;
            if (m.jj0 < G.jp && m.rr0 < rows && jj < G.H) {
                const int b = 2 * jj - L + 1;
                const bool in = __mul24(b, b) + a2 <= rr2;
                const int dk = 16 * k * G.jp;
#pragma unroll
                for (int g = 0; g < IMG; ++g) {
                    if (g >= nimg) break;
                    const float x = X.x[g][1][k][0], y = X.x[g][1][k][1];
                    const float u = in ? fmaxf(x, 0.f) : 0.f, v = in ? fmaxf(y, 0.f) : 0.f;
                    *(LdsF2 *)(uintptr_t)(p0 + dk + g * IB) = f32x2v{u, v};
                    *(LdsF2 *)(uintptr_t)(p1 - dk + g * IB) = f32x2v{v, u};
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < IMG; ++g)
        if (g < nimg && nf[g] != 0.f) bad[g] = 1;
}

// A lane's task here keeps only its row offsets and the LDS address of its
// slot's constants (c = cos theta, r = tan theta, k1 = 2 - 1/c, k2 = 2 - 3c,
// the values of make_task), read once per task and strip: the accumulators of
// two images leave no registers for five constants per task.
struct LaneTask2 {
    int ka;           // byte address of the slot's float4 in the table
    float A3, A3n;
    int rlo, rhi;     // wave-uniform
};

__device__ __forceinline__ LaneTask2 make_task2(const ProjShape &P, const float2 *dtab, int task,
                                                int lane, int kbase) {
    const LaneTask t = make_task(P, dtab, task, lane);
    const int item = task_item(P, task, lane);
    LaneTask2 u;
    u.A3 = t.A3;
    u.A3n = t.A3n;
    u.rlo = t.rlo;
    u.rhi = t.rhi;
    u.ka = kbase + 16 * (item >= 0 ? item / P.L : P.slots);
    return u;
}

// The table: one float4 per slot plus the constants of an empty lane.
template <int NT>
__device__ __forceinline__ void fill_slot_table(const ProjShape &P, const float2 *dtab,
                                                float4 *tab) {
    for (int k = threadIdx.x; k <= P.slots; k += NT) {
        float c = 1.f, r = 0.f, k1 = 1.f;
        if (k < P.slots) {
            const float2 d = dtab[k];
            c = d.x;
            r = -d.y / c;
            k1 = (float)(2.0 - 1.0 / (double)c);
        }
        tab[k] = make_float4(c, r, k1, fmaf(-3.f, c, 2.f));
    }
}

// Accumulate one strip for this wave's tasks and `IMG` images (a missing
// second image reads its zero strips).  Rows pair from even image rows as in
// accumulate_strip.
template <int TPW, int IMG, int IB = kImg2Bytes>
__device__ __forceinline__ void s4_accumulate(const LaneTask2 (&tasks)[TPW], int L,
                                              const float *lds, int i0, int rows,
                                              float (&acc)[IMG][TPW][4], int my_tasks) {
    const float hi3 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)L + 2.f)));
    const int P16 = 16 * s4_positions(L);
    const int lbase = (int)(uintptr_t)(const __attribute__((address_space(3))) float *)lds;
    int s16;
    asm volatile("v_mov_b32 %0, 16" : "=v"(s16));
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t < my_tasks) {  // wave-uniform
            const LaneTask2 tk = tasks[t];
            const f32x4v K = *(const LdsF4 *)(uintptr_t)tk.ka;
            const float c = K.x, tr = K.y, k1 = K.z, k2 = K.w;
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
                const float w0 = fmaf(-c, fr, c);
                const float w1 = fmaf(-c, fabsf(k1 - fr), 1.f);
                const float w2 = __builtin_amdgcn_fmed3f(fmaf(c, fr, k2), 0.f, 1.f);
                const int pa = __mul24(j2, s16) + rbase;
#pragma unroll
                for (int g = 0; g < IMG; ++g) {
                    const f32x4v K0 = *(const LdsF4 *)(uintptr_t)(pa + g * IB);
                    const f32x4v K1 = *(const LdsF4 *)(uintptr_t)(pa + g * IB + 16);
                    const f32x4v K2 = *(const LdsF4 *)(uintptr_t)(pa + g * IB + 32);
                    s[g][0] = fmaf(w2, K2.x, fmaf(w1, K1.x, fmaf(w0, K0.x, s[g][0])));
                    s[g][1] = fmaf(w2, K2.z, fmaf(w1, K1.z, fmaf(w0, K0.z, s[g][1])));
                    s[g][2] = fmaf(w2, K2.y, fmaf(w1, K1.y, fmaf(w0, K0.y, s[g][2])));
                    s[g][3] = fmaf(w2, K2.w, fmaf(w1, K1.w, fmaf(w0, K0.w, s[g][3])));
                }
            };
            int rr = ra;
            if (rr < rb && ((i0 + rr) & 1)) {  // odd first row (wave-uniform)
                row(fmaf((float)(i0 + rr - 1), tr, tk.A3n), lbase + rr * P16);
                ++rr;
            }
            float fi = (float)(i0 + rr);  // even row index, exact in FP32
            for (; rr + 1 < rb; rr += 2, fi += 2.f) {
                const int rbase = lbase + rr * P16;
                row(fmaf(fi, tr, tk.A3), rbase);
                row(fmaf(fi, tr, tk.A3n), rbase + P16);
            }
            if (rr < rb) row(fmaf(fi, tr, tk.A3), lbase + rr * P16);
#pragma unroll
            for (int g = 0; g < IMG; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[g][t][v] = s[g][v];
        }
    }
}

// Projection of `nimg` <= IMG images for the task group starting at task
// tg0 (tasks tg0 + wave + t NW, t < TPW) into the accumulators; lds holds IMG
// strip buffers IB bytes apart, of R rows (R <= s4_rows<NT, KP>(L, IB)), ktab
// (P.slots + 1 entries, 16-byte aligned) the slot constants.  bad[g] is set
// when image g holds a non-finite value.
template <int NT, int TPW, int IMG, int KP = 2, int IB = kImg2Bytes>
__device__ void project_images2(const float *const (&F)[IMG], int nimg, const ProjShape &P,
                                const float2 *__restrict__ dtab, float *lds, float4 *ktab, int R,
                                int tg0, float (&acc)[IMG][TPW][4], int (&bad)[IMG]) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int L = P.L;
    const S4Geo G = s4_geo<NT>(L, R);
#pragma unroll
    for (int g = 0; g < IMG; ++g) {
        bad[g] = 0;
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[g][t][0] = acc[g][t][1] = acc[g][t][2] = acc[g][t][3] = 0.f;
    }
    const int mine = P.ntasks - tg0 - wave;
    const int my_tasks = mine > 0 ? min(TPW, (mine + NW - 1) / NW) : 0;
    const int kbase = (int)(uintptr_t)(__attribute__((address_space(3))) float4 *)ktab;
    LaneTask2 tasks[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) tasks[t] = make_task2(P, dtab, tg0 + wave + t * NW, lane, kbase);
    // the padding positions (and a missing image's strips) stay zero
    __syncthreads();  // the caller may have used the region and the table
    fill_slot_table<NT>(P, dtab, ktab);
    const int used = R * s4_positions(L);  // 16-byte chunks of an image's strips
#pragma unroll
    for (int g = 0; g < IMG; ++g)
        for (int q = threadIdx.x; q < used; q += NT)
            *(float4 *)(lds + g * (IB / 4) + 4 * q) = make_float4(0.f, 0.f, 0.f, 0.f);
    Strip4Regs<IMG, KP> xs;
    s4_load<NT, IMG>(F, nimg, L, 0, G, xs);
    for (int i0 = 0; i0 < L; i0 += R) {
        const int rows = min(R, L - i0);
        __syncthreads();
        s4_store<NT, IMG, KP, IB>(nimg, L, i0, rows, G, xs, lds, bad);
        __syncthreads();
        if (i0 + R < L) s4_load<NT, IMG>(F, nimg, L, i0 + R, G, xs);
        s4_accumulate<TPW, IMG, IB>(tasks, L, lds, i0, rows, acc, my_tasks);
    }
#pragma unroll
    for (int g = 0; g < IMG; ++g) bad[g] = __syncthreads_or(bad[g]);
}

// One image per block in the four-kind strips, any number of task groups
// (each group stages the strips again): strips of R <= strip4_rows_max(L) rows in
// the 64 KiB region at lds, the slot table at ktab; results handed to emit,
// which must not write to the strips or the table.  bad_out: the image holds
// a non-finite value (then nothing is emitted).  Bitwise the sums of
// project_image.
template <int NT, int TPW, typename Emit>
__device__ void project_image4(const float *__restrict__ F, const ProjShape &P,
                               const float2 *__restrict__ dtab, float *lds, float4 *ktab, int R,
                               int &bad_out, Emit emit) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float *const Fa[1] = {F};
    bad_out = 0;
    for (int tg0 = 0; tg0 < P.ntasks; tg0 += NW * TPW) {
        float acc[1][TPW][4];
        int bad[1];
        project_images2<NT, TPW, 1, kImg1Passes>(Fa, 1, P, dtab, lds, ktab, R, tg0, acc, bad);
        if (!bad[0]) emit_outputs<TPW>(P, tg0, wave, NW, lane, acc[0], emit);
        bad_out |= bad[0];
    }
}

}  // namespace sw
