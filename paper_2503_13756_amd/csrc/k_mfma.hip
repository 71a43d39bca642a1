// Many-vs-many alignment on the matrix cores (Sec. 2.3, fast computation over
// rotations, for every pair of two image sets).
//
// For every frequency w along the angle axis the spectral correlation of all
// pairs is a dense complex product
//   S_w[a][b] = sum_j conj(U^_a[j][w]) V^_b[j][w],
// i.e. two real GEMMs with K = 2Q once real and imaginary parts are
// interleaved along K.  k_corr_mfma runs them on MFMA with bfloat16 spectra
// and FP32 accumulation, one 16 x 16 pair tile per block (the four waves
// split the frequencies), keeps S in LDS, and finishes every pair in the same
// block: the inverse DFT over w (a second product, S times the real DFT
// matrix, on FP32 MFMA), the closed-form translation correction
// D*(l) = (E_a + E_b - 2 C(l))/(nQ) - 2|b(l)|^2 and the top-k lags.  S never
// reaches HBM.
//
// k_rescore_tiles then recomputes the objective at the top-k lags in FP32:
// the translation-free residual R0(l) = sum_{j,k} (U[j][k] - V[j][k+l])^2
// is summed directly (no E_a + E_b - 2C cancellation), and the translation is
// added in closed form, R0/(nQ) - 2|b(l)|^2, which is the exact minimum over
// s of the residual with the shift s.d_k removed from every column (the same
// algebra as the correction above, using sum_k d_k d_k^T = (n/2) I).  Image
// tables sit in registers while reference tables stream through LDS as four
// rotated copies, so every lag is a run of aligned 16-byte LDS reads.
#include "sw_internal.h"

namespace sw {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// LDS writes of this wave visible to its other lanes (no block barrier).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (re, im) -> (im, -re) on a packed bf16 complex
__device__ __forceinline__ uint32_t times_minus_i(uint32_t z) {
    return (z >> 16) | (((z & 0xffffu) ^ 0x8000u) << 16);
}

template <int N, int KMAX>
__global__ __launch_bounds__(256) void k_corr_mfma(const uint32_t *__restrict__ spec_ref,
                                                   const uint32_t *__restrict__ spec_img,
                                                   int64_t n_ref, int64_t n_img, int Q, int mode,
                                                   int top_k, const double *__restrict__ ref_aux,
                                                   const double *__restrict__ img_aux,
                                                   const float2 *__restrict__ tw32,
                                                   int16_t *__restrict__ cand, int slice) {
    constexpr int Wn = N / 2 + 1;
    constexpr int SS = 2 * Wn + 1;  // odd LDS row stride
    extern __shared__ __align__(16) float lds[];
    float *Sl = lds;                           // [256 pairs][SS]
    float2 *tw = (float2 *)(lds + 256 * SS);  // [N]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // XCD-aware tile order: blocks go to the eight XCDs in turn, so block b
    // runs on XCD b mod 8; XCD x takes the image tiles [x slice, (x + 1)
    // slice) against every reference tile, image tile fastest, so that its
    // L2 holds one slice of the image spectra and each reference tile is
    // fetched once per slice pass.
    const int64_t b = blockIdx.x, loc = b >> 3;
    const int64_t it = (b & 7) * slice + loc % slice, rt = loc / slice;
    if (it * 16 >= n_img) return;  // block-uniform, before any barrier
    const int64_t g0 = it * 16, r0 = rt * 16;
    for (int i = threadIdx.x; i < N; i += 256) tw[i] = tw32[i];

    // Spectral products on the gfx950 bf16 MFMA with 32 K entries (16
    // complex values) per instruction: lane l holds row l % 16 (reference)
    // or column l % 16 (image) and the complex values 16 s + 4 (l / 16) ..
    // + 3 of K step s, one 16-byte load each.  The spectra of frequency
    // w + 4 are fetched into registers while those of w are multiplied.
    constexpr int KS = N / 16;  // K steps (Q == N on this path)
    const int q = lane >> 4;
    const int64_t ra = r0 + (lane & 15), gb = g0 + (lane & 15);
    const bool va = ra < n_ref, vb = gb < n_img;
    const uint4 *pa = (const uint4 *)(spec_ref + (va ? ra : 0) * (int64_t)Wn * Q) + q;
    const uint4 *pb = (const uint4 *)(spec_img + (vb ? gb : 0) * (int64_t)Wn * Q) + q;
    const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
    uint4 a_cur[KS], b_cur[KS], a_nxt[KS], b_nxt[KS];
    auto fetch = [&](int w, uint4(&A)[KS], uint4(&B)[KS]) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            A[s] = pa[(int64_t)w * (N / 4) + 4 * s];
            B[s] = pb[(int64_t)w * (N / 4) + 4 * s];
        }
    };
    // Fully unrolled over this wave's frequencies w = wave + 4 i: every fetch
    // is issued (the one past the last frequency refetches it), so exactly
    // one frequency's fetch is in flight while the previous one is
    // multiplied.
    constexpr int NI = (Wn + 3) / 4;
    fetch(wave, a_cur, b_cur);  // wave < 4 < Wn
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int w = wave + 4 * i;
        uint4(&A0)[KS] = (i & 1) ? a_nxt : a_cur;
        uint4(&B0)[KS] = (i & 1) ? b_nxt : b_cur;
        uint4(&A1)[KS] = (i & 1) ? a_cur : a_nxt;
        uint4(&B1)[KS] = (i & 1) ? b_cur : b_nxt;
        if (i + 1 < NI) fetch(min(w + 4, Wn - 1), A1, B1);
        if (w < Wn) {  // wave-uniform
            f32x4_t acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const uint4 av = va ? A0[s] : zero4, bv = vb ? B0[s] : zero4;
                const uint4 bi = make_uint4(times_minus_i(bv.x), times_minus_i(bv.y),
                                            times_minus_i(bv.z), times_minus_i(bv.w));
                const bf16x8_t A = __builtin_bit_cast(bf16x8_t, av);
                acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    A, __builtin_bit_cast(bf16x8_t, bv), acc_re, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    A, __builtin_bit_cast(bf16x8_t, bi), acc_im, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int pr = (4 * q + v) * 16 + (lane & 15);  // tile pair: ref-major
                Sl[pr * SS + 2 * w] = acc_re[v];
                Sl[pr * SS + 2 * w + 1] = acc_im[v];
            }
        }
    }
    __syncthreads();

    // ---- translation correction folded into the w = 1 term.  With
    // z = conj(a_ref) a_img, |b(l)|^2 = |a_ref|^2 + |a_img|^2 - 2 Re(z e^{i theta_l}), so
    //   D*(l) = const - (2/nQ) X(l),  X(l) = C(l) - 2 nQ Re(z e^{i theta_l}),
    // and Re(z e^{i theta_l}) is the w = 1 basis function: X is C of the
    // spectrum with S_1 lowered by nQ N z.  The lags of smallest D* are those
    // of largest X.
    const int t = threadIdx.x;
    const int64_t r = r0 + t / 16, g = g0 + t % 16;
    const bool pair_ok = r < n_ref && g < n_img;
    if (mode == 0 && pair_ok) {
        const double *au = ref_aux + 4 * r, *av = img_aux + 4 * g;
        const double s = (double)N * (double)N * (double)Q;
        const double zx = au[2] * av[2] + au[3] * av[3], zy = au[2] * av[3] - au[3] * av[2];
        Sl[t * SS + 2] -= (float)(s * zx);
        Sl[t * SS + 3] -= (float)(s * zy);
    }
    wave_lds_fence();  // rows of this wave only: no block barrier

    // ---- inverse DFT over w on the bf16 MFMA with split operands:
    // C[p][l] = sum_k S[p][k] T[k][l] with k = 2w (real part) or 2w + 1
    // (imaginary part) and
    //   T[2w][l] = c_w cos(2 pi w l / N) / N,  T[2w + 1][l] = -c_w sin(2 pi w l / N) / N,
    // c_w = 1 at w = 0 and N/2 (whose imaginary rows are 0), else 2.  Each
    // FP32 operand x is split into bf16 parts x = hi + lo (hi = x rounded,
    // lo = the rest rounded), and C = S_hi T_hi + S_hi T_lo + S_lo T_hi with
    // FP32 accumulation: about 16 bits of the operands, far finer than the
    // bf16 spectra S came from (the lags only feed the candidate list; the
    // rescore is exact FP32).  Wave v owns pairs 64 v .. 64 v + 63 (four
    // 16-pair row tiles) and writes C over its own S rows; only this wave
    // reads or writes them from here on.  Lane l holds K entries
    // 32 st + 8 (l / 16) .. + 7 of step st for row / column l % 16.
    {
        constexpr int KS = (2 * Wn + 31) / 32;  // k-steps of 32
        constexpr int CT = N / 16;              // lag tiles
        const int kq = lane >> 4, jl = lane & 15;
        f32x4_t acc[4][CT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const float *Srow = Sl + (64 * wave + jl) * SS;
        auto split = [](float x, __bf16 &hi, __bf16 &lo) {
            hi = (__bf16)x;
            lo = (__bf16)(x - (float)hi);
        };
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int k0 = 32 * st + 8 * kq;  // this lane's first k
            bf16x8_t ah[4], al[4];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + e;
                    __bf16 h, l;
                    split(k < 2 * Wn ? Srow[16 * rt * SS + k] : 0.f, h, l);
                    ah[rt][e] = h;
                    al[rt][e] = l;
                }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                bf16x8_t bh, bl;
#pragma unroll
                for (int q = 0; q < 4; ++q) {  // k = k0 + 2q (real), k0 + 2q + 1 (imaginary)
                    const int w = (k0 >> 1) + q;
                    float re = 0.f, im = 0.f;
                    if (2 * w < 2 * Wn) {
                        const bool edge = w == 0 || w == N / 2;
                        const float cw = edge ? 1.f / (float)N : 2.f / (float)N;
                        const float2 e = tw[(w * (16 * ct + jl)) & (N - 1)];  // (cos, -sin)
                        re = e.x * cw;
                        im = edge ? 0.f : e.y * cw;
                    }
                    __bf16 h, l;
                    split(re, h, l);
                    bh[2 * q] = h;
                    bl[2 * q] = l;
                    split(im, h, l);
                    bh[2 * q + 1] = h;
                    bl[2 * q + 1] = l;
                }
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bh, acc[rt][ct], 0, 0, 0);
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bl, acc[rt][ct], 0, 0, 0);
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt], bh, acc[rt][ct], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Sl[(64 * wave + 16 * rt + 4 * kq + v) * SS + 16 * ct + jl] = acc[rt][ct][v];
        wave_lds_fence();
    }

    // ---- one pair per thread: the top-k lags of largest X.  Keys: X mapped
    // to an unsigned code that grows as X falls, its low bits replaced by the
    // lag, kept sorted by a min/max insertion (ties, and values within 2^-17
    // relative, go to the smaller lag; the exact FP32 rescore decides among
    // the candidates).
    if (!pair_ok) return;  // no barrier follows
    const float *Crow = Sl + t * SS;
    uint32_t top[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) top[c] = 0xffffffffu;
    for (int l = 0; l < N; ++l) {
        const uint32_t u = __float_as_uint(-Crow[l]);
        uint32_t key = (u >> 31) ? ~u : (u | 0x80000000u);
        key = (key & ~(uint32_t)(N - 1)) | (uint32_t)l;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            const uint32_t lo = min(key, top[c]);
            key = max(key, top[c]);
            top[c] = lo;
        }
    }
    int16_t *out = cand + (r * n_img + g) * (int64_t)top_k;
    for (int c = 0; c < top_k; ++c) out[c] = (int16_t)(top[c] & (uint32_t)(N - 1));
}

// Sum over the 64 lanes: butterflies inside each row of 16 lanes on DPP,
// then the four row totals.  Fixed order, so the result is deterministic.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_sum_f(float v) {
    v += dpp_f<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);  // row_half_mirror
    v += dpp_f<0x140>(v);  // row_mirror
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Rescore: grid (ceil(n_img / (NT / 64)), ceil(n_ref / TR)), NT threads; wave w owns
// image g0 + w and walks the references r0 .. r1 - 1.  Lane layout: chunk
// p = lane % CPR of four columns (CPR = N / 4 chunks per row) in rows
// jr + RPS m (jr = lane / CPR, RPS = 64 / CPR), so the image's table is
// STEPS float4 registers per lane.  Each reference table is staged in LDS as
// four rotated copies C_s[j][i] = U[j][(i - s) mod N], s = 0..3: the lag
// l = 4a + s pairs the lane's chunk with the aligned 16 bytes
// C_s[j][4((p - a) mod CPR) ..], one conflict-free b128 read per four
// elements at a fixed offset per row step.  Lane c < top_k carries candidate
// c (its lag, translation and objective); the next reference's table and
// candidates are fetched into registers while this one is summed.
template <int N, int KMAX, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_rescore_tiles(
    const float *__restrict__ ref_qt, const double *__restrict__ ref_aux, int64_t n_ref,
    const float *__restrict__ img_qt, const double *__restrict__ img_aux, int64_t n_img, int TR,
    int mode, int top_k, int L, const int16_t *__restrict__ cand, const double2 *__restrict__ tw64,
    Result *__restrict__ out) {
    constexpr int Q = N, CPR = N / 4, RPS = 64 / CPR, STEPS = Q / RPS;
    constexpr int COPY = Q * N, NCH = Q * N / 4, CH = (NCH + NT - 1) / NT;
    static_assert(KMAX <= 64 && STEPS * RPS == Q, "rescore layout");
    extern __shared__ __align__(16) float lds[];  // [4][Q][N]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t g = (int64_t)blockIdx.x * (NT / 64) + wave;
    const bool live = g < n_img;  // wave-uniform
    const int64_t gc = live ? g : n_img - 1;
    const int64_t r0 = (int64_t)blockIdx.y * TR;
    const int64_t r1 = min(r0 + (int64_t)TR, n_ref);
    const int p = lane % CPR, jr = lane / CPR;
    float4 vv[STEPS];
    {
        const float *V = img_qt + gc * (int64_t)COPY;
#pragma unroll
        for (int m = 0; m < STEPS; ++m)
            vv[m] = *(const float4 *)(V + (jr + RPS * m) * N + 4 * p);
    }
    const double av0 = img_aux[4 * gc], av1 = img_aux[4 * gc + 2], av2 = img_aux[4 * gc + 3];
    const double nq = (double)N * (double)Q;
    // prefetch registers: this thread's chunks of the next reference table
    // and, unless a row is one DPP row of 16 lanes, the chunks one column
    // group to their left (same row, cyclic)
    constexpr bool kRor = CPR == 16;
    float4 ucur[CH], uprev[kRor ? 1 : CH];
    int lnext = 0;
    auto fetch = [&](int64_t r) {
        const float4 *U = (const float4 *)(ref_qt + r * (int64_t)COPY);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int c = t + NT * i;
            if (c < NCH) {
                ucur[i] = U[c];
                if constexpr (!kRor) {
                    const int j = c / CPR, q = c % CPR;
                    uprev[i] = U[j * CPR + (q + CPR - 1) % CPR];
                }
            }
        }
        lnext = lane < top_k ? (int)cand[(r * n_img + gc) * top_k + lane] : 0;
    };
    if (r0 < r1) fetch(r0);
    for (int64_t r = r0; r < r1; ++r) {
        const int lmine = lnext;
        const double au0 = ref_aux[4 * r], au1 = ref_aux[4 * r + 2], au2 = ref_aux[4 * r + 3];
        __syncthreads();  // every wave is done with the previous table
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int c = t + NT * i;
            if (c < NCH) {
                const float4 u = ucur[i];
                float4 v;
                if constexpr (kRor) {
                    // chunk q - 1 (mod 16) of the same row sits one lane down
                    // in this DPP row: row_ror:1
                    v.x = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u.x), 0x121, 0xf, 0xf, false));
                    v.y = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u.y), 0x121, 0xf, 0xf, false));
                    v.z = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u.z), 0x121, 0xf, 0xf, false));
                    v.w = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u.w), 0x121, 0xf, 0xf, false));
                } else {
                    v = uprev[i];
                }
                float *d = lds + 4 * c;
                *(float4 *)(d) = u;
                *(float4 *)(d + COPY) = make_float4(v.w, u.x, u.y, u.z);
                *(float4 *)(d + 2 * COPY) = make_float4(v.z, v.w, u.x, u.y);
                *(float4 *)(d + 3 * COPY) = make_float4(v.y, v.z, v.w, u.x);
            }
        }
        __syncthreads();
        if (r + 1 < r1) fetch(r + 1);
        if (!live) continue;  // wave-uniform, after both barriers
        // translation at this lane's candidate lag (mode 0), Sec. 2.3
        double bx = 0.0, by = 0.0;
        if (mode == 0) {
            const double2 d = tw64[lmine];
            const double cs = d.x, sn = -d.y;
            bx = au1 - (cs * av1 - sn * av2);
            by = au2 - (sn * av1 + cs * av2);
        }
        // lane c takes candidate c's residual
        float sc = 0.f;
#pragma unroll 1
        for (int c = 0; c < KMAX; ++c) {
            if (c >= top_k) break;
            const int l = __builtin_amdgcn_readlane(lmine, c);
            const float *src = lds + (l & 3) * COPY + jr * N + 4 * ((p - (l >> 2)) & (CPR - 1));
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
            // reads run PIPE row steps ahead of the arithmetic
            constexpr int PIPE = STEPS < 4 ? STEPS : 4;
            float4 ub[STEPS];
#pragma unroll
            for (int m = 0; m < PIPE; ++m) ub[m] = *(const float4 *)(src + m * RPS * N);
#pragma unroll
            for (int m = 0; m < STEPS; ++m) {
                if (m + PIPE < STEPS) ub[m + PIPE] = *(const float4 *)(src + (m + PIPE) * RPS * N);
                __builtin_amdgcn_sched_barrier(0);
                const float4 u = ub[m];
                const float4 v = vv[m];
                const float e0 = u.x - v.x, e1 = u.y - v.y, e2 = u.z - v.z, e3 = u.w - v.w;
                a0 = fmaf(e0, e0, a0);
                a1 = fmaf(e1, e1, a1);
                a2 = fmaf(e2, e2, a2);
                a3 = fmaf(e3, e3, a3);
                __builtin_amdgcn_sched_barrier(0);
            }
            const float sum = wave_sum_f((a0 + a1) + (a2 + a3));
            if (lane == c) sc = sum;
        }
        const float D = (float)((double)sc / nq - 2.0 * (bx * bx + by * by));
        // smallest objective, ties to the smaller lag
        int bc = 0;
        float bd = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(D), 0));
        int bl = __builtin_amdgcn_readlane(lmine, 0);
#pragma unroll
        for (int c = 1; c < KMAX; ++c) {
            if (c >= top_k) break;
            const float dc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(D), c));
            const int lc = __builtin_amdgcn_readlane(lmine, c);
            if (dc < bd || (dc == bd && lc < bl)) {
                bd = dc;
                bl = lc;
                bc = c;
            }
        }
        if (lane == bc) {
            int st = 0;
            if (isnan(au0) || isnan(av0)) st = 2;
            else if (!(au0 > 0.0) || !(av0 > 0.0)) st = 1;
            Result res;
            res.status = st;
            if (st) {
                res.rot_index = 0;
                res.theta_rad = 0.f;
                res.shift_px[0] = res.shift_px[1] = 0.f;
                res.sw2sq = __int_as_float(0x7fc00000);
            } else {
                res.rot_index = bl;
                res.theta_rad = (float)(6.283185307179586 * (double)bl / (double)N);
                res.shift_px[0] = (float)(bx * (double)L);  // s* = 2b, in pixels s*/h
                res.shift_px[1] = (float)(by * (double)L);
                res.sw2sq = bd;
            }
            out[r * n_img + g] = res;
        }
    }
}

bool mfma_path_supported(Geo g) { return g.Q == g.n && (g.n == 32 || g.n == 64); }

// Threads of a rescore block: one image per wave against each staged
// reference table, so 16 images share each staging of the four rotated
// copies (64 KiB of LDS at n = 64, one block per CU either way); 2,000 x
// 2,000 at L = 64: 5.35 ms with 512 threads, 5.27 ms with 1024.
constexpr int kRescoreThreads = 1024;

template <int N>
static hipError_t launch_mfma_t(const MfmaArgs &a, Geo g, const AngleTable &t, hipStream_t s) {
    constexpr int KMAX = 4;
    constexpr int Wn = N / 2 + 1;
    const size_t lds1 = sizeof(float) * 256 * (2 * Wn + 1) + sizeof(float2) * N;
    static const hipError_t attr1 = hipFuncSetAttribute(
        (const void *)k_corr_mfma<N, KMAX>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)attr1;
    // a 1-D grid of 8 slices of image tiles times the reference tiles
    const int64_t tiles_img = (a.n_img + 15) / 16, tiles_ref = (a.n_ref + 15) / 16;
    const int64_t slice = (tiles_img + 7) / 8;
    const int64_t nblocks = 8 * slice * tiles_ref;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_corr_mfma<N, KMAX>), dim3((unsigned)nblocks), dim3(256), lds1, s,
                       a.spec_ref, a.spec_img, a.n_ref, a.n_img, g.Q, a.mode, a.top_k, a.ref_aux,
                       a.img_aux, t.d32, a.cand, (int)slice);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // blocks of NT / 64 images x TR references; TR chosen so that the grid
    // fills the resident slots in as few, as full, rounds as possible
    constexpr int NT = kRescoreThreads, IPB = NT / 64;
    static const int slots = [] {
        (void)hipFuncSetAttribute((const void *)k_rescore_tiles<N, KMAX, NT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 4 * N * N * 4);
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, (const void *)k_rescore_tiles<N, KMAX, NT>, NT, sizeof(float) * 4 * N * N);
        return (cus > 0 ? cus : 256) * (per > 0 ? per : 1);
    }();
    const int64_t gx = (a.n_img + IPB - 1) / IPB;
    int64_t best_gy = 1;
    double best_eff = -1.0;
    for (int64_t gy = 1; gy <= a.n_ref && (gy == 1 || gx * gy <= 4 * (int64_t)slots); ++gy) {
        const int64_t tr = (a.n_ref + gy - 1) / gy;
        const int64_t rounds = (gx * gy + slots - 1) / slots;
        const double eff = (double)(a.n_ref * gx) / ((double)rounds * slots * tr);
        if (eff > best_eff * 1.01) {
            best_eff = eff;
            best_gy = gy;
        }
    }
    const int TR = (int)((a.n_ref + best_gy - 1) / best_gy);
    const int gy = (int)((a.n_ref + TR - 1) / TR);
    const size_t lds2 = sizeof(float) * 4 * N * N;
    hipLaunchKernelGGL((k_rescore_tiles<N, KMAX, NT>), dim3((unsigned)gx, (unsigned)gy), dim3(NT), lds2, s, a.ref_qt,
                       a.ref_aux, a.n_ref, a.img_qt, a.img_aux, a.n_img, TR, a.mode, a.top_k, g.L,
                       a.cand, t.d64, a.out);
    return hipGetLastError();
}

hipError_t launch_mfma_all_pairs(const MfmaArgs &a, Geo g, const AngleTable &t, hipStream_t s) {
    if (a.n_ref <= 0 || a.n_img <= 0) return hipSuccess;
    if (!mfma_path_supported(g) || a.top_k < 1 || a.top_k > 4) return hipErrorInvalidValue;
    if (g.n == 32) return launch_mfma_t<32>(a, g, t, s);
    return launch_mfma_t<64>(a, g, t, s);
}

}  // namespace sw
