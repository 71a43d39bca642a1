// Pair alignment specialised for n = 128 angles (Sec. 2.3, fast computation
// over rotations; translation by Thm 3.2 as in align_dev.h), with the angle
// FFTs held in registers instead of LDS passes.
//
// Packed rows: table rows 2p and 2p+1 of the image form the complex row
// z_p[k] = V[2p][k] + i V[2p+1][k].  Eight lanes transform one packed row:
// lane l holds z[l + 8m], m = 0..15, does a 16-point DFT over m in registers,
// multiplies by w128^(l t), and after a transpose through LDS (within the
// eight lanes) lane l' holds, for t0 = 2l' + tau (tau = 0, 1), the values
// Y[0..7][t0] and does an 8-point DFT over them:
//   Z_p[t0 + 16 s] = sum_l w8^(l s) w128^(l t0) sum_m w16^(m t0) z[l + 8m].
// The spectral dot S(w) = sum_j conj(U^_j(w)) V^_j(w) needs the spectra of
// the two real rows, A = (Z(w) + conj(Z(-w)))/2 and B = (Z(w) - conj(Z(-w)))/2i;
// with alpha_p(w) = (conj(Ue) - i conj(Uo))/2 and beta_p(w) = (conj(Ue) +
// i conj(Uo))/2 from the reference spectra Ue = U^_{2p}, Uo = U^_{2p+1},
//   S(w) = sum_p Z_p(w) alpha_p(w) + conj(Z_p(n - w)) beta_p(w),
// so every Z_p(f) makes one complex multiply-add: into S(f) with alpha for
// f < 64, into S(128 - f) with conj and beta for f > 64 (both for f = 0, 64).
// The per-reference coefficients are laid out in the lane order, 16 complex
// per lane and packed row.
#pragma once
#include <type_traits>

#include "align_dev.h"

namespace sw {

constexpr int kA128Slots = 128;  // coefficients per packed row (8 lanes x 16)

// Coefficient `slot` of packed row p (slot < 128: lane slot l'*16 + tau*8 + s;
// 128: beta_p(0); 129: alpha_p(64)) from the FP32 spectrum spec[65][Q] of U.
__device__ __forceinline__ float2 gamma128_coef(const float2 *__restrict__ spec, int Q, int p,
                                                int slot) {
    int w;
    bool use_beta;
    if (slot < kA128Slots) {
        const int lp = slot >> 4, tau = (slot >> 3) & 1, s = slot & 7;
        const int f = 2 * lp + tau + 16 * s;
        use_beta = s >= 4;
        w = use_beta ? 128 - f : f;
    } else {
        use_beta = slot == kA128Slots;
        w = use_beta ? 0 : 64;
    }
    const float2 *sp = spec + (int64_t)w * Q + 2 * p;
    const float2 ue = sp[0], uo = sp[1];
    return use_beta ? make_float2(0.5f * (ue.x + uo.y), 0.5f * (uo.x - ue.y))
                    : make_float2(0.5f * (ue.x - uo.y), -0.5f * (ue.y + uo.x));
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * conj-free constant (c, s): forward twiddle values are (cos, -sin)
__device__ __forceinline__ float2 ctw(float2 a, float c, float s) {
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// In-place forward DFT-4 of (a0, a1, a2, a3).
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - i t3
    a3 = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + i t3
}

// Forward DFT-16 of x[0..15]; the result Y[t] is returned in x[t].
__device__ __forceinline__ void dft16(float2 (&x)[16]) {
    // m = 4a + b: DFT-4 over a for each b (result for c in x[b + 4c])
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4(x[b], x[b + 4], x[b + 8], x[b + 12]);
    // twiddles w16^(b c)
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f;
    constexpr float h = 0.70710678118654752f;
    x[1 + 4] = ctw(x[1 + 4], c1, -s1);   // b=1 c=1: w^1
    x[1 + 8] = ctw(x[1 + 8], h, -h);     // b=1 c=2: w^2
    x[1 + 12] = ctw(x[1 + 12], s1, -c1); // b=1 c=3: w^3
    x[2 + 4] = ctw(x[2 + 4], h, -h);     // b=2 c=1: w^2
    x[2 + 8] = make_float2(x[2 + 8].y, -x[2 + 8].x);  // b=2 c=2: w^4 = -i
    x[2 + 12] = ctw(x[2 + 12], -h, -h);  // b=2 c=3: w^6
    x[3 + 4] = ctw(x[3 + 4], s1, -c1);   // b=3 c=1: w^3
    x[3 + 8] = ctw(x[3 + 8], -h, -h);    // b=3 c=2: w^6
    x[3 + 12] = ctw(x[3 + 12], -c1, s1); // b=3 c=3: w^9
    // DFT-4 over b for each c: register 4c + d then holds Y[c + 4d]
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4(x[4 * c], x[4 * c + 1], x[4 * c + 2], x[4 * c + 3]);
    float2 y[16];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = 0; d < 4; ++d) y[c + 4 * d] = x[4 * c + d];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = y[t];
}

// Forward DFT-8 of u[0..7] in natural order.
__device__ __forceinline__ void dft8(float2 (&u)[8]) {
    float2 e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    float2 o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    constexpr float h = 0.70710678118654752f;
    o1 = ctw(o1, h, -h);
    o2 = make_float2(o2.y, -o2.x);
    o3 = ctw(o3, -h, -h);
    u[0] = cadd(e0, o0);
    u[4] = csub(e0, o0);
    u[1] = cadd(e1, o1);
    u[5] = csub(e1, o1);
    u[2] = cadd(e2, o2);
    u[6] = csub(e2, o2);
    u[3] = cadd(e3, o3);
    u[7] = csub(e3, o3);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kA128Stride = 18;  // complex per lane row of the transpose buffer (16 + pad)
constexpr int kA128VRow = 132;   // floats per staged table row (128 + pad)
// The per-wave layout: the two rows of a packed pair contiguous (as in the
// table, so that one 1 KiB memory-to-LDS copy stages a pair), pairs 264
// floats apart (the 8 groups' reads still fall in distinct banks).
constexpr int kA128PairStride = 264;

struct A128NoHook {
    __device__ void operator()() const {}
};

// Spectrum of the packed row of lane group `grp`, whose two table rows are
// staged at varea + 2 grp kA128VRow (rows kA128VRow floats apart), or with
// PAIRED at varea + grp kA128PairStride (rows 128 floats apart): lane l8
// ends with Z[2 l8 + tau + 16 s] in u_tau[s].  buf: the group's 8 x
// kA128Stride transpose buffer (it may overlap the staged rows: they are read
// first).  after(): called once the wave's last LDS read of the staged rows
// and the buffer is done (the wave may refill them).  Wave-synchronous.
template <bool PAIRED = false, typename After = A128NoHook>
__device__ __forceinline__ void a128_row_spectrum(const float *varea, float2 *buf,
                                                  const float2 *tw, int grp, int l8,
                                                  float2 (&u0)[8], float2 (&u1)[8],
                                                  After after = After()) {
    constexpr int n = 128;
    constexpr int kRow2 = PAIRED ? 128 : kA128VRow;
    float2 x[16];
    const float *zr = varea + (PAIRED ? grp * kA128PairStride : 2 * grp * kA128VRow) + l8;
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = make_float2(zr[8 * m], zr[kRow2 + 8 * m]);
    wave_lds_sync();
    dft16(x);
    // l8 t < n: the twiddle addresses are formed here from an opaque copy of
    // l8 rather than kept live across the caller's loop (15 registers)
    int lt = l8;
    asm volatile("" : "+v"(lt));
#pragma unroll
    for (int t = 1; t < 16; ++t) x[t] = cmul(x[t], tw[lt * t]);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        *(float4 *)(buf + l8 * kA128Stride + 2 * k) =
            make_float4(x[2 * k].x, x[2 * k].y, x[2 * k + 1].x, x[2 * k + 1].y);
    wave_lds_sync();
#pragma unroll
    for (int l = 0; l < 8; ++l) {
        const float4 q = *(const float4 *)(buf + l * kA128Stride + 2 * l8);
        u0[l] = make_float2(q.x, q.y);
        u1[l] = make_float2(q.z, q.w);
    }
    wave_lds_sync();
    after();
    dft8(u0);
    dft8(u1);
}

// Spectral dot of packed row p into the lane's 16 slots (slot tau 8 + s holds
// frequency f = 2 l8 + tau + 16 s; f > 64 accumulates conj(Z) beta into
// S(128 - f)); lane 0 of the group also adds conj(Z(0)) beta_p(0) and
// Z(64) alpha_p(64).  BF16: operands rounded to bfloat16 first (a compile-time
// choice: as a run-time flag the compiler computes the roundings on both paths
// and selects, about half the VALU work of a pass).
template <bool BF16>
__device__ __forceinline__ void a128_dot(float2 (&acc)[16], const float2 (&u0)[8],
                                         const float2 (&u1)[8], const float2 *__restrict__ G,
                                         const float2 *__restrict__ GX, int p, int l8) {
    const float4 *gp = (const float4 *)(G + (int64_t)p * kA128Slots + l8 * 16);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float4 gq = gp[k];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int slot = 2 * k + h, tau = slot >> 3, s = slot & 7;
            float2 z = tau ? u1[s] : u0[s];
            float2 c = h ? make_float2(gq.z, gq.w) : make_float2(gq.x, gq.y);
            if constexpr (BF16) {
                z = bf16r2(z);
                c = bf16r2(c);
            }
            if (s >= 4) z.y = -z.y;  // conj(Z) beta for f > 64
            acc[slot].x += z.x * c.x - z.y * c.y;
            acc[slot].y += z.x * c.y + z.y * c.x;
        }
    }
    if (l8 == 0) {
        // f = 0 also takes conj(Z) beta_p(0); f = 64 also takes Z alpha_p(64)
        float2 z0 = u0[0], z4 = u0[4];
        float2 c0 = GX[2 * p], c4 = GX[2 * p + 1];
        if constexpr (BF16) {
            z0 = bf16r2(z0);
            z4 = bf16r2(z4);
            c0 = bf16r2(c0);
            c4 = bf16r2(c4);
        }
        acc[0].x += z0.x * c0.x + z0.y * c0.y;
        acc[0].y += z0.x * c0.y - z0.y * c0.x;
        acc[4].x += z4.x * c4.x - z4.y * c4.y;
        acc[4].y += z4.x * c4.y + z4.y * c4.x;
    }
}

// Slot of frequency f in a lane group's buffer of partial sums: lane
// (f mod 16) / 2, entry (f mod 2) 8 + f / 16.
__device__ __forceinline__ int a128_slot(int f) {
    return ((f & 15) >> 1) * kA128Stride + (f & 1) * 8 + (f >> 4);
}

// LDS of one block of the n = 128 alignment.
template <int NT>
struct A128Lds {
    float2 tw[128];
    __attribute__((aligned(16))) float2 xb[NT / 64 * 8 * 8 * kA128Stride];
    float2 S[65];
    double D[128];
    float red[NT / 64][kMaxTopK];
    int cand[kMaxTopK];
    float2 cs[kMaxTopK];  // 2 b(l) of every candidate, FP32
};

// One pair, whole block.  status != 0 writes the failed record.
struct A128Job {
    const float *U, *V;          // [Q][128] tables
    const double *au, *av;       // aux
    const float2 *G, *GX;        // coefficients of U: [Q/2][128], [Q/2][2]
    const float2 *d32;           // angle table, n = 128
    const double2 *d64;
    Result *res;
    float *curve;                // nullable, [128]
    int Q, L, mode, bf16, top_k, status;
};

// BF16 is job.bf16 as a compile-time choice.
template <int NT, bool BF16>
__device__ void align128_pair(const A128Job &job, A128Lds<NT> &sm) {
    constexpr int n = 128, NW = NT / 64, NG = NW * 8;  // lane groups per block
    float2 *tw = sm.tw, *xb = sm.xb, *S = sm.S;
    double *D = sm.D;
    float (*red)[kMaxTopK] = sm.red;
    int *cand = sm.cand;
    float2 *cs = sm.cs;
    const int Q = job.Q, P2 = Q / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l8 = lane & 7, grp = lane >> 3;
    __syncthreads();  // the previous job of this block may still read LDS
    if (job.status) {
        if (threadIdx.x == 0) {
            job.res->rot_index = 0;
            job.res->theta_rad = 0.f;
            job.res->shift_px[0] = job.res->shift_px[1] = 0.f;
            job.res->sw2sq = __int_as_float(0x7fc00000);
            job.res->status = job.status;
        }
        if (job.curve)
            for (int l = threadIdx.x; l < n; l += NT) job.curve[l] = __int_as_float(0x7fc00000);
        return;
    }
    for (int i = threadIdx.x; i < n; i += NT) tw[i] = job.d32[i];
    __syncthreads();
    const float *U = job.U, *V = job.V;
    const float2 *G = job.G, *GX = job.GX;
    const double *au = job.au, *av = job.av;
    const double2 *tw64 = job.d64;
    Result *res = job.res;
    float *curve = job.curve;

    // --- angle FFTs of the packed rows and the spectral dot
    float2 acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = make_float2(0.f, 0.f);
    float2 *buf = xb + (wave * 8 + grp) * 8 * kA128Stride;
    // the wave stages the 16 table rows of its 8 packed rows into its part of
    // the transpose buffer with coalesced 16-byte loads (rows kA128VRow
    // floats apart, the two rows of a packed row adjacent), and each lane
    // then reads its strided elements from LDS
    float *varea = (float *)(xb + wave * 8 * 8 * kA128Stride);
    const int iters = (P2 + NG - 1) / NG;
    for (int it = 0; it < iters; ++it) {
        const int pbase = wave * 8 + it * NG;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int q = lane + 64 * i;          // 16-byte chunk, 32 per table row
            const int row = q >> 5, c4 = q & 31;  // row = 2 (group) + (odd row)
            const int gp = pbase + (row >> 1);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gp < P2) v = *(const float4 *)(V + (int64_t)(2 * gp + (row & 1)) * n + 4 * c4);
            *(float4 *)(varea + row * kA128VRow + 4 * c4) = v;
        }
        wave_lds_sync();
        const int p = pbase + grp;
        float2 u0[8], u1[8];
        a128_row_spectrum(varea, buf, tw, grp, l8, u0, u1);
        // an opaque copy of l8: the coefficient address is formed per
        // iteration rather than held (or spilled) across the loop
        int l8o = l8;
        asm volatile("" : "+v"(l8o));
        if (p < P2) a128_dot<BF16>(acc, u0, u1, G, GX, p, l8o);
    }
    // --- partial sums of every lane group to LDS, then S(w) for w = 0..64
#pragma unroll
    for (int k = 0; k < 8; ++k)
        *(float4 *)(buf + l8 * kA128Stride + 2 * k) =
            make_float4(acc[2 * k].x, acc[2 * k].y, acc[2 * k + 1].x, acc[2 * k + 1].y);
    __syncthreads();
    // slot holding frequency f in the group buffer: lane (f mod 16) / 2,
    // entry (f mod 2) * 8 + f / 16
    for (int t = threadIdx.x; t < 65 * 8; t += NT) {
        const int w = t >> 3, part = t & 7;
        const int fa = w < 64 ? w : 64;
        const int ia = ((fa & 15) >> 1) * kA128Stride + (fa & 1) * 8 + (fa >> 4);
        const int fb = 128 - w;  // second contribution for 1 <= w <= 63
        const int ib = ((fb & 15) >> 1) * kA128Stride + (fb & 1) * 8 + (fb >> 4);
        float2 s = make_float2(0.f, 0.f);
        for (int gg = part * (NG / 8); gg < (part + 1) * (NG / 8); ++gg) {
            const float2 *gb = xb + gg * 8 * kA128Stride;
            s = cadd(s, gb[ia]);
            if (w >= 1 && w <= 63) s = cadd(s, gb[ib]);
        }
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            s.x += __shfl_xor(s.x, off, 64);
            s.y += __shfl_xor(s.y, off, 64);
        }
        if (part == 0) S[w] = s;
    }
    __syncthreads();
    // The transpose buffer is free from here on: the rescore's first chunk of
    // V rows is copied into it straight from memory to LDS (1 KiB per wave
    // instruction, no registers) while the lags are scored.
    constexpr int RC = (NG * 8 * kA128Stride * 2) / n >= 128 ? 128 : 64;  // rows per chunk
    static_assert(RC * n <= NG * 8 * kA128Stride * 2, "chunk fits the buffer");
    {
        const int rows0 = Q < RC ? Q : RC;
        const int segs = rows0 * n / 256;  // 1 KiB segments (n = 128: two rows each)
        for (int q = wave; q < segs; q += NW)
            __builtin_amdgcn_global_load_lds(
                (const void *)(job.V + 256 * q + 4 * lane),
                (__attribute__((address_space(3))) void *)((float *)xb + 256 * q), 16, 0, 0);
    }

    // --- inverse transform over w, translation correction, objective per lag.
    // Lags l and l + 64 share every twiddle (e^{2 pi i w 64 / n} = (-1)^w):
    // a task sums the even and the odd w of its quarter apart and gives both.
    const double nq = (double)n * (double)Q;
    for (int t = threadIdx.x; t < n * 2; t += NT) {
        const int l = t >> 2, part = t & 3;
        float se = 0.f, so = 0.f;
        const int w0 = 1 + 16 * part, w1 = part == 3 ? 63 : w0 + 15;  // w0 odd
        int m = (w0 * l) & (n - 1);
        for (int w = w0; w <= w1; w += 2) {
            const float2 t1 = tw[m];
            so += S[w].x * t1.x + S[w].y * t1.y;  // Re(S e^{+2 pi i w l / n})
            m = (m + l) & (n - 1);
            if (w + 1 <= w1) {
                const float2 t2 = tw[m];
                se += S[w + 1].x * t2.x + S[w + 1].y * t2.y;
            }
            m = (m + l) & (n - 1);
        }
        float sum = se + so, sum64 = se - so;
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        sum64 += __shfl_xor(sum64, 1, 64);
        sum64 += __shfl_xor(sum64, 2, 64);
        if (part < 2) {  // part 0: lag l, part 1: lag l + 64
            const int lp = l + 64 * part;
            const float a0 = S[0].x + ((l & 1) ? -S[n / 2].x : S[n / 2].x);
            const double Cl = ((double)a0 + 2.0 * (double)(part ? sum64 : sum)) / (double)n;
            double d = (au[1] + av[1] - 2.0 * Cl) / nq;
            if (job.mode == 0) {
                const double2 b = trans_moment(au, av, tw64[lp]);
                d -= 2.0 * (b.x * b.x + b.y * b.y);
            }
            D[lp] = d;
            if (curve) curve[lp] = (float)d;
        }
    }
    __syncthreads();

    // --- top-K lags (wave 0; ties to the smaller lag)
    const int K = job.top_k;
    if (wave == 0) {
        double v0 = D[lane], v1 = D[lane + 64];
        for (int c = 0; c < K; ++c) {
            double v = v0;
            int i = lane;
            argmin_merge(v, i, v1, lane + 64);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double v2 = __shfl_xor(v, off, 64);
                const int i2 = __shfl_xor(i, off, 64);
                argmin_merge(v, i, v2, i2);
            }
            if (lane == 0) cand[c] = i;
            if (i == lane) v0 = __builtin_inf();
            if (i == lane + 64) v1 = __builtin_inf();
        }
    }
    __syncthreads();

    // --- FP32 rescore of the candidates: direct residual sum.  V is staged
    // through LDS in chunks of rows (coalesced 16-byte loads), so
    // that the rotated reads V[j][(k + l) mod n] are LDS reads; consecutive
    // lanes take consecutive k.  Two candidates per pass; the per-wave
    // partial sums of every chunk are added in chunk order.
    if (threadIdx.x < K) {
        const int c = threadIdx.x;
        double2 b = make_double2(0.0, 0.0);
        if (job.mode == 0) b = trans_moment(au, av, tw64[cand[c]]);
        cs[c] = make_float2((float)(2.0 * b.x), (float)(2.0 * b.y));
    }
    if (lane < K) red[wave][lane] = 0.f;
    float *vl = (float *)xb;
    for (int j0 = 0; j0 < Q; j0 += RC) {
        const int rows = Q - j0 < RC ? Q - j0 : RC;
        if (j0 == 0) {
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copy above has landed
        } else {
            __syncthreads();
            for (int q = threadIdx.x; q < rows * (n / 4); q += NT)
                *(float4 *)(vl + 4 * q) = *(const float4 *)(V + (int64_t)j0 * n + 4 * q);
        }
        __syncthreads();
        // a thread keeps one column k (NT is a multiple of n) and walks
        // rows kRows apart, so the angle, the shift terms and the rotated
        // column offsets are per-thread constants
        constexpr int kRows = NT / n;
        const int k = threadIdx.x & (n - 1), jt = threadIdx.x / n;
        const float2 dk = tw[k];
        const float *Uc = U + (int64_t)j0 * n + k;
        for (int c0 = 0; c0 < K; c0 += 2) {
            const float *va = vl + ((k + cand[c0]) & (n - 1));
            const float sa = cs[c0].x * dk.x + cs[c0].y * dk.y;
            float pa = 0.f;
            if (c0 + 1 < K) {  // two candidates per pass (block-uniform)
                const int c1 = c0 + 1;
                const float *vb = vl + ((k + cand[c1]) & (n - 1));
                const float sb = cs[c1].x * dk.x + cs[c1].y * dk.y;
                float pb = 0.f;
#pragma unroll 8
                for (int jr = jt; jr < rows; jr += kRows) {
                    const float u = Uc[jr * n];
                    const float da = u - va[jr * n] - sa;
                    const float db = u - vb[jr * n] - sb;
                    pa += da * da;
                    pb += db * db;
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    pa += __shfl_xor(pa, off, 64);
                    pb += __shfl_xor(pb, off, 64);
                }
                if (lane == 0) {
                    red[wave][c0] += pa;
                    red[wave][c1] += pb;
                }
            } else {  // the last candidate of an odd count alone
#pragma unroll 8
                for (int jr = jt; jr < rows; jr += kRows) {
                    const float da = Uc[jr * n] - va[jr * n] - sa;
                    pa += da * da;
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) pa += __shfl_xor(pa, off, 64);
                if (lane == 0) red[wave][c0] += pa;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best_l = 0;
        float best = 0.f, bsx = 0.f, bsy = 0.f;
        for (int c = 0; c < K; ++c) {
            float s = 0.f;
            for (int w = 0; w < NW; ++w) s += red[w][c];
            const float v = s / (float)nq;
            if (c == 0 || v < best || (v == best && cand[c] < best_l)) {
                best = v;
                best_l = cand[c];
                bsx = cs[c].x;
                bsy = cs[c].y;
            }
        }
        const float L = (float)job.L;
        res->rot_index = best_l;
        res->theta_rad = (float)(6.283185307179586 * (double)best_l / (double)n);
        res->shift_px[0] = bsx * 0.5f * L;
        res->shift_px[1] = bsy * 0.5f * L;
        res->sw2sq = best;
        res->status = 0;
    }
}

// The same alignment with one pair per wave: the transforms and the spectral
// dot as in align128_pair, the eight lane groups' partial sums added through
// the wave's LDS, lags l and l + 64 per lane, the top K lags by a butterfly
// over the lanes, and the FP32 rescore from image rows copied to LDS eight
// at a time, double-buffered.
// No block barrier: the waves of a block run independent pairs.  xb: the
// wave's kA128WaveElems float2 of LDS; tw: the angle table in LDS.
constexpr int kA128WaveElems = 8 * 8 * kA128Stride;

__device__ void align128_wave(const A128Job &job, float2 *xb, const float2 *tw) {
    constexpr int n = 128;
    const int Q = job.Q, P2 = Q / 2;
    // an opaque copy of the lane index: in a persistent caller, the per-lane
    // addresses derived from it are formed per pair instead of being kept
    // live (or spilled) across pairs
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int l8 = lane & 7, grp = lane >> 3;
    if (job.status) {
        if (lane == 0) {
            job.res->rot_index = 0;
            job.res->theta_rad = 0.f;
            job.res->shift_px[0] = job.res->shift_px[1] = 0.f;
            job.res->sw2sq = __int_as_float(0x7fc00000);
            job.res->status = job.status;
        }
        if (job.curve) {
            job.curve[lane] = __int_as_float(0x7fc00000);
            job.curve[lane + 64] = __int_as_float(0x7fc00000);
        }
        return;
    }
    const float *U = job.U, *V = job.V;
    const double *au = job.au, *av = job.av;
    float *varea = (float *)xb;
    float2 *buf = xb + grp * 8 * kA128Stride;

    // 8 packed pairs of table rows [r0, r0 + 16) of V into varea by
    // memory-to-LDS copies, one 1 KiB copy per pair (the pair's two rows are
    // contiguous in the table and in varea, pairs kA128PairStride apart).
    // Pairs past Q copy the last pair again: their transforms are computed
    // and never used.  The next stage's copies are issued as soon as the
    // current rows and the transpose buffer have been read, so that they fly
    // during the last transforms and the spectral dot.
    auto stage = [&](int r0) {
        // the copies write the LDS behind the ds_read path: every read of
        // the area (the staged rows and the transpose buffers overlap it)
        // must have returned first, or a copy that lands early overwrites
        // rows still to be read
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int r = min(r0 + 2 * i, Q - 2);  // Q is even
            __builtin_amdgcn_global_load_lds(
                (const void *)(V + (int64_t)r * n + 4 * lane),
                (__attribute__((address_space(3))) void *)(varea + i * kA128PairStride), 16, 0,
                0);
        }
    };

    // --- angle FFTs of the packed rows and the spectral dot
    float2 acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = make_float2(0.f, 0.f);
    stage(0);
    auto pass = [&](auto bf16) {
        for (int pbase = 0; pbase < P2; pbase += 8) {
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this stage's copies have landed
            wave_lds_sync();
            const int p = pbase + grp;
            float2 u0[8], u1[8];
            a128_row_spectrum<true>(varea, buf, tw, grp, l8, u0, u1, [&]() {
                if (pbase + 8 < P2) stage(2 * (pbase + 8));
            });
            if (p < P2) a128_dot<decltype(bf16)::value>(acc, u0, u1, job.G, job.GX, p, l8);
        }
    };
    if (job.bf16)
        pass(std::true_type{});
    else
        pass(std::false_type{});

    // --- the groups' partial sums, then S(w): lane t forms T(t) and
    // T(t + 64), S(w) = T(w) + T(128 - w) for 1 <= w <= 63, S(0) = T(0),
    // S(64) = T(64)
#pragma unroll
    for (int k = 0; k < 8; ++k)
        *(float4 *)(buf + l8 * kA128Stride + 2 * k) =
            make_float4(acc[2 * k].x, acc[2 * k].y, acc[2 * k + 1].x, acc[2 * k + 1].y);
    wave_lds_sync();
    float2 t1 = make_float2(0.f, 0.f), t2 = make_float2(0.f, 0.f);
    {
        const int i1 = a128_slot(lane), i2 = a128_slot(lane + 64);
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            t1 = cadd(t1, xb[g * 8 * kA128Stride + i1]);
            t2 = cadd(t2, xb[g * 8 * kA128Stride + i2]);
        }
    }
    const float ox = __shfl(t2.x, (64 - lane) & 63, 64), oy = __shfl(t2.y, (64 - lane) & 63, 64);
    wave_lds_sync();
    float2 *S = xb;  // 65 values
    S[lane] = lane == 0 ? t1 : make_float2(t1.x + ox, t1.y + oy);
    if (lane == 0) S[64] = t2;
    wave_lds_sync();

    // --- inverse transform for lags l = lane and l + 64 (e^{2 pi i w 64 / n}
    // = (-1)^w), translation correction, objective
    const int l = lane;
    float se = 0.f, so = 0.f;
    {
        int m = l;  // w l mod n for w = 1
        for (int w = 1; w < 64; w += 2) {
            const float2 a = tw[m], sa = S[w];
            so += sa.x * a.x + sa.y * a.y;  // Re(S e^{+2 pi i w l / n})
            m = (m + l) & (n - 1);
            if (w < 63) {
                const float2 b = tw[m], sb = S[w + 1];
                se += sb.x * b.x + sb.y * b.y;
            }
            m = (m + l) & (n - 1);
        }
    }
    const double nq = (double)n * (double)Q;
    double dl[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int lp = l + 64 * h;
        const float a0 = S[0].x + ((l & 1) ? -S[n / 2].x : S[n / 2].x);
        const double Cl = ((double)a0 + 2.0 * (double)(h ? se - so : se + so)) / (double)n;
        double d = (au[1] + av[1] - 2.0 * Cl) / nq;
        if (job.mode == 0) {
            const double2 b = trans_moment(au, av, job.d64[lp]);
            d -= 2.0 * (b.x * b.x + b.y * b.y);
        }
        dl[h] = d;
        if (job.curve) job.curve[lp] = (float)d;
    }

    // --- top-K lags (ties to the smaller lag), the same on every lane
    const int K = job.top_k;
    int cand[kMaxTopK];
    {
        double v0 = dl[0], v1 = dl[1];
#pragma unroll
        for (int c = 0; c < kMaxTopK; ++c) {
            cand[c] = 0;
            if (c < K) {
                double v = v0;
                int i = lane;
                argmin_merge(v, i, v1, lane + 64);
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const double v2 = __shfl_xor(v, off, 64);
                    const int i2 = __shfl_xor(i, off, 64);
                    argmin_merge(v, i, v2, i2);
                }
                cand[c] = __builtin_amdgcn_readfirstlane(i);
                if (i == lane) v0 = __builtin_inf();
                if (i == lane + 64) v1 = __builtin_inf();
            }
        }
    }

    // --- FP32 rescore of the candidates: direct residual sum, lane columns
    // k = 2 lane, 2 lane + 1
    float2 cs[kMaxTopK];
    float sh0[kMaxTopK], sh1[kMaxTopK], part[kMaxTopK];
    const int k0 = 2 * lane;
    const float2 dk0 = tw[k0], dk1 = tw[k0 + 1];
#pragma unroll
    for (int c = 0; c < kMaxTopK; ++c) {
        cs[c] = make_float2(0.f, 0.f);
        if (c < K && job.mode == 0) {
            const double2 b = trans_moment(au, av, job.d64[cand[c]]);
            cs[c] = make_float2((float)(2.0 * b.x), (float)(2.0 * b.y));
        }
        sh0[c] = cs[c].x * dk0.x + cs[c].y * dk0.y;
        sh1[c] = cs[c].x * dk1.x + cs[c].y * dk1.y;
        part[c] = 0.f;
    }
    // rows in chunks of 8, double-buffered in the wave's LDS (rows of n
    // floats) by memory-to-LDS copies: the next chunk's rows and the
    // reference rows it needs are in flight while the current chunk is summed
    float *vb0 = (float *)xb, *vb1 = vb0 + 8 * n;
    auto issue = [&](int r0, float *dst, float2 (&u)[8]) {
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): earlier reads of dst have returned
#pragma unroll
        for (int q = 0; q < 4; ++q)  // 1 KiB = two rows per copy (Q is even)
            if (r0 + 2 * q < Q)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(V + (int64_t)(r0 + 2 * q) * n + 4 * lane),
                    (__attribute__((address_space(3))) void *)(dst + 2 * q * n), 16, 0, 0);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            u[r] = r0 + r < Q ? *(const float2 *)(U + (int64_t)(r0 + r) * n + k0)
                              : make_float2(0.f, 0.f);
    };
    auto sum_chunk = [&](int r0, const float *vb, const float2 (&u)[8]) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r0 + r < Q) {
                const float *vr = vb + r * n;
#pragma unroll
                for (int c = 0; c < kMaxTopK; ++c) {
                    if (c < K) {
                        const float d0 = u[r].x - vr[(k0 + cand[c]) & (n - 1)] - sh0[c];
                        const float d1 = u[r].y - vr[(k0 + 1 + cand[c]) & (n - 1)] - sh1[c];
                        part[c] = fmaf(d0, d0, part[c]);
                        part[c] = fmaf(d1, d1, part[c]);
                    }
                }
            }
        }
    };
    float2 ua[8], ub[8];
    wave_lds_sync();  // S is no longer read
    issue(0, vb0, ua);
    for (int r0 = 0; r0 < Q; r0 += 16) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): chunk r0 has landed
        wave_lds_sync();
        if (r0 + 8 < Q) issue(r0 + 8, vb1, ub);
        sum_chunk(r0, vb0, ua);
        if (r0 + 8 >= Q) break;
        __builtin_amdgcn_s_waitcnt(0x0F70);  // chunk r0 + 8 has landed
        wave_lds_sync();
        if (r0 + 16 < Q) issue(r0 + 16, vb0, ua);
        sum_chunk(r0 + 8, vb1, ub);
    }
    int best_l = 0;
    float best = 0.f, bsx = 0.f, bsy = 0.f;
#pragma unroll
    for (int c = 0; c < kMaxTopK; ++c) {
        if (c < K) {
            float t = part[c];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
            const float v = t / (float)nq;
            if (c == 0 || v < best || (v == best && cand[c] < best_l)) {
                best = v;
                best_l = cand[c];
                bsx = cs[c].x;
                bsy = cs[c].y;
            }
        }
    }
    if (lane == 0) {
        const float Lf = (float)job.L;
        Result *res = job.res;
        res->rot_index = best_l;
        res->theta_rad = (float)(6.283185307179586 * (double)best_l / (double)n);
        res->shift_px[0] = bsx * 0.5f * Lf;
        res->shift_px[1] = bsy * 0.5f * Lf;
        res->sw2sq = best;
        res->status = 0;
    }
}

}  // namespace sw
