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
// block: the inverse DFT over w (even/odd split), the closed-form translation
// correction D*(l) = (E_a + E_b - 2 C(l))/(nQ) - 2|b(l)|^2 and the top-k lags.
// S never reaches HBM.
//
// k_rescore_tiles then recomputes the objective at the top-k lags in FP32:
// the translation-free residual R0(l) = sum_{j,k} (U[j][k] - V[j][k+l])^2
// is summed directly (no E_a + E_b - 2C cancellation), and the translation is
// added in closed form, R0/(nQ) - 2|b(l)|^2, which is the exact minimum over
// s of the residual with the shift s.d_k removed from every column (the same
// algebra as the correction above, using sum_k d_k d_k^T = (n/2) I).  V tables
// of TG images sit in registers while reference tables stream through LDS as
// duplicated rows, so every lag is a fixed-offset LDS read.
#include "sw_internal.h"

namespace sw {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x4_t as_bf16x4(uint32_t lo, uint32_t hi) {
    bf16x4_t v;
    v[0] = (short)(lo & 0xffffu);
    v[1] = (short)(lo >> 16);
    v[2] = (short)(hi & 0xffffu);
    v[3] = (short)(hi >> 16);
    return v;
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
                                                   int16_t *__restrict__ cand) {
    constexpr int Wn = N / 2 + 1;
    constexpr int SS = 2 * Wn + 1;  // odd LDS row stride
    extern __shared__ __align__(16) float lds[];
    float *Sl = lds;                           // [256 pairs][SS]
    float2 *tw = (float2 *)(lds + 256 * SS);  // [N]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * 16, r0 = (int64_t)blockIdx.y * 16;
    for (int i = threadIdx.x; i < N; i += 256) tw[i] = tw32[i];

    const int q = lane >> 4;
    const int64_t ra = r0 + (lane & 15), gb = g0 + (lane & 15);
    const bool va = ra < n_ref, vb = gb < n_img;
    const uint32_t *pa = spec_ref + (va ? ra : 0) * (int64_t)Wn * Q;
    const uint32_t *pb = spec_img + (vb ? gb : 0) * (int64_t)Wn * Q;
    for (int w = wave; w < Wn; w += 4) {
        f32x4_t acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
        const uint32_t *ar = pa + (int64_t)w * Q;
        const uint32_t *br = pb + (int64_t)w * Q;
        for (int s = 0; s < Q / 8; ++s) {
            const int j = 8 * s + 2 * q;  // two complex values = four K entries
            uint2 av = make_uint2(0u, 0u), bv = make_uint2(0u, 0u);
            if (va) av = *(const uint2 *)(ar + j);
            if (vb) bv = *(const uint2 *)(br + j);
            const bf16x4_t A = as_bf16x4(av.x, av.y);
            const bf16x4_t B = as_bf16x4(bv.x, bv.y);
            const bf16x4_t Bi = as_bf16x4(times_minus_i(bv.x), times_minus_i(bv.y));
            acc_re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bi, acc_im, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int pr = (4 * q + v) * 16 + (lane & 15);  // tile pair: ref-major
            Sl[pr * SS + 2 * w] = acc_re[v];
            Sl[pr * SS + 2 * w + 1] = acc_im[v];
        }
    }
    __syncthreads();

    // ---- one pair per thread: inverse DFT over w, correction, top-k
    const int t = threadIdx.x;
    const int64_t r = r0 + t / 16, g = g0 + t % 16;
    if (r >= n_ref || g >= n_img) return;  // no barrier follows
    float S[2 * Wn];
#pragma unroll
    for (int i = 0; i < 2 * Wn; ++i) S[i] = Sl[t * SS + i];
    const double *au = ref_aux + 4 * r, *av = img_aux + 4 * g;
    const float Esum = (float)(au[1] + av[1]);
    const float aux_ = (float)au[2], auy = (float)au[3], avx = (float)av[2], avy = (float)av[3];
    const float inv_nq = 1.f / ((float)N * (float)Q);
    float bd[KMAX];
    int bl[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        bd[c] = __builtin_inff();
        bl[c] = 0x7fff;
    }
    auto consider = [&](int l, float Cl) {
        float d = (Esum - 2.f * Cl) * inv_nq;
        if (mode == 0) {
            const float2 e = tw[l];  // (cos, -sin)
            const float bx = aux_ - (e.x * avx + e.y * avy);
            const float by = auy - (-e.y * avx + e.x * avy);
            d -= 2.f * (bx * bx + by * by);
        }
        int li = l;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < top_k) {
                const bool better = d < bd[c] || (d == bd[c] && li < bl[c]);
                if (better) {
                    const float td = bd[c];
                    const int tl = bl[c];
                    bd[c] = d;
                    bl[c] = li;
                    d = td;
                    li = tl;
                }
            }
        }
    };
    const float s0 = S[0], sh = S[2 * (N / 2)];
    const float sgn_half = ((N / 2) & 1) ? -1.f : 1.f;
    for (int l = 0; l < N / 2; ++l) {
        float ev = 0.f, od = 0.f;
#pragma unroll
        for (int w = 1; w < N / 2; ++w) {
            const float2 e = tw[(w * l) & (N - 1)];
            const float term = S[2 * w] * e.x + S[2 * w + 1] * e.y;  // Re(S e^{+i 2 pi w l/n})
            if (w & 1) od += term;
            else ev += term;
        }
        const float alt = (l & 1) ? -sh : sh;
        const float c_lo = (s0 + alt + 2.f * (ev + od)) / (float)N;
        const float c_hi = (s0 + sgn_half * alt + 2.f * (ev - od)) / (float)N;
        consider(l, c_lo);
        consider(l + N / 2, c_hi);
    }
    int16_t *out = cand + (r * n_img + g) * (int64_t)top_k;
    for (int c = 0; c < top_k; ++c) out[c] = (int16_t)bl[c];
}

// Rescore: grid (ceil(n_img / 8), ceil(n_ref / TR)), 256 threads.  Wave w
// holds the V tables of images g0 + 2w and g0 + 2w + 1 in registers: lane l
// owns elements e = l + 64 m (m < EPT), i.e. column k = l % N and rows
// j = l / N + m (64 / N) (N divides 64).  Reference tables stream through LDS.
template <int N, int KMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_rescore_tiles(
    const float *__restrict__ ref_qt, const double *__restrict__ ref_aux, int64_t n_ref,
    const float *__restrict__ img_qt, const double *__restrict__ img_aux, int64_t n_img, int TR,
    int mode, int top_k, int L, const int16_t *__restrict__ cand, const double2 *__restrict__ tw64,
    Result *__restrict__ out) {
    constexpr int Q = N;
    constexpr int EPT = Q * N / 64;
    constexpr int RS = 64 / N;  // rows per element step
    extern __shared__ __align__(16) float lds[];
    float *U2 = lds;  // [Q][2N]: each row stored twice
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * 8 + 2 * wave;
    const int64_t r0 = (int64_t)blockIdx.y * TR;
    const int64_t r1 = min((int64_t)r0 + TR, n_ref);
    const int kcol = lane % N, jrow = lane / N;
    float vv[2][EPT];
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
        const int64_t g = g0 + gi < n_img ? g0 + gi : n_img - 1;
        const float *V = img_qt + g * (int64_t)Q * N;
#pragma unroll
        for (int m = 0; m < EPT; ++m) vv[gi][m] = V[lane + 64 * m];
    }
    const int base = jrow * 2 * N + kcol + N;  // U2 index of (jrow, kcol) shifted by N
    const double nq = (double)N * (double)Q;
    for (int64_t r = r0; r < r1; ++r) {
        __syncthreads();
        const float *U = ref_qt + r * (int64_t)Q * N;
        for (int e = t; e < Q * N; e += 256) {
            const float u = U[e];
            const int j = e / N, k = e % N;
            U2[j * 2 * N + k] = u;
            U2[j * 2 * N + k + N] = u;
        }
        __syncthreads();
        const double *au = ref_aux + 4 * r;
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            const int64_t g = g0 + gi;
            if (g >= n_img) continue;  // wave-uniform
            const int64_t p = r * n_img + g;
            float best = 0.f;
            int bl = 0;
            double bxb = 0.0, byb = 0.0;
            const double *av = img_aux + 4 * g;
            for (int c = 0; c < top_k; ++c) {
                const int l = cand[p * top_k + c];
                // element (j, k) of V pairs with U[j][k - l]
                const float *u2 = U2 + base - l;
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < EPT; ++m) {
                    const float e = u2[m * RS * 2 * N] - vv[gi][m];
                    acc = fmaf(e, e, acc);
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
                double bx = 0.0, by = 0.0;
                if (mode == 0) {
                    const double2 d = tw64[l];
                    const double cs = d.x, sn = -d.y;
                    bx = au[2] - (cs * av[2] - sn * av[3]);
                    by = au[3] - (sn * av[2] + cs * av[3]);
                }
                const float D = (float)((double)acc / nq - 2.0 * (bx * bx + by * by));
                if (c == 0 || D < best || (D == best && l < bl)) {
                    best = D;
                    bl = l;
                    bxb = bx;
                    byb = by;
                }
            }
            if (lane == 0) {
                int st = 0;
                if (isnan(au[0]) || isnan(av[0])) st = 2;
                else if (!(au[0] > 0.0) || !(av[0] > 0.0)) st = 1;
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
                    res.shift_px[0] = (float)(bxb * (double)L);  // s* = 2b, in pixels s*/h
                    res.shift_px[1] = (float)(byb * (double)L);
                    res.sw2sq = best;
                }
                out[p] = res;
            }
        }
    }
}

bool mfma_path_supported(Geo g) { return g.Q == g.n && (g.n == 32 || g.n == 64); }

template <int N>
static hipError_t launch_mfma_t(const MfmaArgs &a, Geo g, const AngleTable &t, hipStream_t s) {
    constexpr int KMAX = 4;
    constexpr int Wn = N / 2 + 1;
    const size_t lds1 = sizeof(float) * 256 * (2 * Wn + 1) + sizeof(float2) * N;
    static const hipError_t attr1 = hipFuncSetAttribute(
        (const void *)k_corr_mfma<N, KMAX>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)attr1;
    dim3 grid1((unsigned)((a.n_img + 15) / 16), (unsigned)((a.n_ref + 15) / 16));
    hipLaunchKernelGGL((k_corr_mfma<N, KMAX>), grid1, dim3(256), lds1, s, a.spec_ref, a.spec_img,
                       a.n_ref, a.n_img, g.Q, a.mode, a.top_k, a.ref_aux, a.img_aux, t.d32, a.cand);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gx = (int)((a.n_img + 7) / 8);
    int gy = (1024 + gx - 1) / gx;  // about four blocks per CU in total
    if (gy > a.n_ref) gy = (int)a.n_ref;
    if (gy < 1) gy = 1;
    const int TR = (int)((a.n_ref + gy - 1) / gy);
    gy = (int)((a.n_ref + TR - 1) / TR);
    const size_t lds2 = sizeof(float) * g.Q * 2 * N;
    hipLaunchKernelGGL((k_rescore_tiles<N, KMAX>), dim3(gx, gy), dim3(256), lds2, s, a.ref_qt,
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
