// Fourier-slice projector (Sec. 2.2: the 1-D Fourier transform of the line
// projection at angle theta is the central slice of the image's 2-D Fourier
// transform; Sec. 2.3 computes the slices with a NUFFT and returns to the
// detector with a 1-D inverse DFT).  The discretisation is that of the
// appendix's fixed-angle error theorem with NUFFT precision: slice
// frequencies k pi, k = -M .. M-1 (L = 2M), and the trigonometric polynomial
// with coefficients yhat_k / 2 sampled at the detector bin centres.
//
// One block per image slot of a persistent grid; per image:
//  1. rows: the pixel masses (positive part inside the disk, exactly as for
//     the line sum) divided by the kernel's Fourier transform at their
//     centred index, zero-padded to Nf = 2L and transformed along x; two
//     real rows share one complex FFT.  The half spectrum v <= Nf/2 goes to
//     the slot's scratch (R).
//  2. columns: the same transform along y for every v <= Nf/2 (B, the
//     oversampled spectrum; the other half is its conjugate mirror).
//  3. slices: every slice point k pi d_theta (theta in [0, pi), k = 0..M) is
//     interpolated from B with a separable exponential-of-semicircle kernel
//     of width kW, phase-shifted to the pixel centres and multiplied by the
//     transform of one pixel cell; the coefficients of two slices are packed
//     into one complex L-point inverse FFT (both results are real), scaled by
//     h/2, clipped at zero and written with their theta + pi mirror.
// The FFTs are radix-2 Stockham transforms in LDS over a batch of sequences.
#include "sw_internal.h"

namespace sw {

namespace {

constexpr int kFftFloats2 = 2048;  // float2 per FFT work buffer

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ bool in_disk_f(int L, int i, int j) {
    const int a = 2 * j - L + 1, b = 2 * i - L + 1, r = L - 2;
    return a * a + b * b <= r * r;
}

// cnt transforms of length 2^lg held at a[f << lg .. ]; b is a work buffer of
// the same size.  tw[k] = exp(-2 pi i k / 2^lg), k < 2^(lg-1); inv selects
// the conjugate twiddles (exp(+2 pi i ...)).  Inputs must be visible to the
// whole block on entry; returns the buffer holding the (naturally ordered)
// result, visible to the whole block.
template <int NT>
__device__ float2 *fft_batch(float2 *a, float2 *b, int lg, int cnt, const float2 *tw, bool inv) {
    const int half = 1 << (lg - 1), total = cnt * half;
    for (int s = 0; s < lg; ++s) {
        const int Ns = 1 << s;
        __syncthreads();
        for (int idx = threadIdx.x; idx < total; idx += NT) {
            const int f = idx >> (lg - 1), j = idx & (half - 1);
            const float2 *src = a + (f << lg);
            float2 *dst = b + (f << lg);
            const float2 v0 = src[j];
            float2 t = tw[(j & (Ns - 1)) << (lg - 1 - s)];
            if (inv) t.y = -t.y;
            const float2 v1 = cmul(src[j + half], t);
            const int o = ((j & ~(Ns - 1)) << 1) + (j & (Ns - 1));
            dst[o] = make_float2(v0.x + v1.x, v0.y + v1.y);
            dst[o + Ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
        }
        float2 *x = a;
        a = b;
        b = x;
    }
    __syncthreads();
    return a;
}

// Slice value yhat at k pi d from the oversampled spectrum B [Nf][H].
__device__ float2 slice_point(const float2 *__restrict__ B, int Nf, int H, int L, double dx,
                              double dy, int k, float beta) {
    const double scale = (double)Nf / (double)L;
    const double gx = k * dx * scale, gy = k * dy * scale;  // fine-grid coordinates
    const int vx0 = (int)floor(gx - 0.5 * kFourierW) + 1;
    const int uy0 = (int)floor(gy - 0.5 * kFourierW) + 1;
    const float fx = (float)(gx - vx0), fy = (float)(gy - uy0);  // in [kW/2 - 1, kW/2)
    float wx[kFourierW], wy[kFourierW];
#pragma unroll
    for (int c = 0; c < kFourierW; ++c) {
        const float tx = 2.f * (fx - (float)c) / (float)kFourierW;
        const float ty = 2.f * (fy - (float)c) / (float)kFourierW;
        wx[c] = fabsf(tx) < 1.f ? expf(beta * (sqrtf(1.f - tx * tx) - 1.f)) : 0.f;
        wy[c] = fabsf(ty) < 1.f ? expf(beta * (sqrtf(1.f - ty * ty) - 1.f)) : 0.f;
    }
    const int hm = Nf >> 1, msk = Nf - 1;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < kFourierW; ++a) {
        const int u = (uy0 + a) & msk, um = (Nf - u) & msk;
        float2 ra = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < kFourierW; ++c) {
            const int v = (vx0 + c) & msk;
            float2 bv;
            if (v <= hm) {
                bv = B[u * H + v];
            } else {  // conjugate mirror of the stored half
                bv = B[um * H + (Nf - v)];
                bv.y = -bv.y;
            }
            ra.x = fmaf(wx[c], bv.x, ra.x);
            ra.y = fmaf(wx[c], bv.y, ra.y);
        }
        acc.x = fmaf(wy[a], ra.x, acc.x);
        acc.y = fmaf(wy[a], ra.y, acc.y);
    }
    // pixel centres sit half a pixel off the centred integer grid, and the
    // cell transform sinc(xi_x h/2) sinc(xi_y h/2) with xi h/2 = k pi d / L
    const double pi = 3.141592653589793238462643383279502884;
    const double ang = -pi * k * (dx + dy) / L;
    const double ax = pi * k * dx / L, ay = pi * k * dy / L;
    const double sx = ax == 0.0 ? 1.0 : sin(ax) / ax, sy = ay == 0.0 ? 1.0 : sin(ay) / ay;
    const float2 ph = make_float2((float)(cos(ang) * sx * sy), (float)(sin(ang) * sx * sy));
    return cmul(acc, ph);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_fourier(const float *__restrict__ img, int64_t N,
                                                FourierShape S, FourierTabs T,
                                                const double2 *__restrict__ d64,
                                                float2 *__restrict__ scratch, float *__restrict__ pmf) {
    extern __shared__ __align__(16) float2 lds2[];
    __shared__ int sbad;
    const int L = S.L, M = L >> 1, n = S.n, Nf = S.Nf, H = S.H, lgNf = S.lgNf, lgL = S.lgL;
    const float h = 2.f / (float)L;
    float2 *fa = lds2, *fb = lds2 + kFftFloats2;
    float2 *Y = fb + kFftFloats2;                      // [slices][M + 1]
    float2 *twf = Y + (2 * kFftFloats2 / L) * (M + 1);  // [Nf / 2]
    float2 *twl = twf + (Nf >> 1);                      // [L / 2]
    float2 *shf = twl + (L >> 1);                       // [L]
    float *corr = (float *)(shf + L);                   // [L]
    for (int t = threadIdx.x; t < (Nf >> 1); t += NT) twf[t] = T.twf[t];
    for (int t = threadIdx.x; t < (L >> 1); t += NT) twl[t] = T.twl[t];
    for (int t = threadIdx.x; t < L; t += NT) {
        shf[t] = T.shift[t];
        corr[t] = T.corr[t];
    }
    float2 *R = scratch + (size_t)blockIdx.x * (size_t)(L + Nf) * H;  // [L][H]
    float2 *B = R + (size_t)L * H;                                      // [Nf][H]
    const int GR = kFftFloats2 >> lgNf;  // transforms of length Nf per round
    const int GS = kFftFloats2 >> lgL;   // transforms of length L per round (two slices each)
    for (int64_t g = blockIdx.x; g < N; g += gridDim.x) {
        const float *F = img + g * (int64_t)L * L;
        __syncthreads();  // previous image done with sbad and the buffers
        if (threadIdx.x == 0) sbad = 0;
        int bad = 0;
        // 1. rows, two per transform
        for (int p0 = 0; p0 < M; p0 += GR) {
            const int cnt = min(GR, M - p0);
            __syncthreads();
            for (int idx = threadIdx.x; idx < (cnt << lgNf); idx += NT) {
                const int f = idx >> lgNf, q = idx & (Nf - 1);
                const int j = (q < (Nf >> 1) ? q : q - Nf) + M;
                float2 z = make_float2(0.f, 0.f);
                if (j >= 0 && j < L) {
                    const int i = 2 * (p0 + f);
                    const float x0 = F[(int64_t)i * L + j], x1 = F[(int64_t)(i + 1) * L + j];
                    if (!isfinite(x0) || !isfinite(x1)) bad = 1;
                    const float cj = corr[j];
                    z.x = (in_disk_f(L, i, j) && x0 > 0.f) ? x0 * (corr[i] * cj) : 0.f;
                    z.y = (in_disk_f(L, i + 1, j) && x1 > 0.f) ? x1 * (corr[i + 1] * cj) : 0.f;
                }
                fa[idx] = z;
            }
            const float2 *X = fft_batch<NT>(fa, fb, lgNf, cnt, twf, false);
            for (int idx = threadIdx.x; idx < cnt * H; idx += NT) {
                const int f = idx / H, v = idx - f * H;
                const float2 zv = X[(f << lgNf) + v], zc = X[(f << lgNf) + ((Nf - v) & (Nf - 1))];
                const int i = 2 * (p0 + f);
                // Z = X_i + i X_{i+1}: X_i[v] = (Z[v] + conj Z[-v]) / 2,
                // X_{i+1}[v] = (Z[v] - conj Z[-v]) / (2 i)
                R[(size_t)i * H + v] = make_float2(0.5f * (zv.x + zc.x), 0.5f * (zv.y - zc.y));
                R[(size_t)(i + 1) * H + v] = make_float2(0.5f * (zv.y + zc.y), -0.5f * (zv.x - zc.x));
            }
        }
        if (bad) sbad = 1;
        // 2. columns
        for (int v0 = 0; v0 < H; v0 += GR) {
            const int cnt = min(GR, H - v0);
            __syncthreads();  // R written; work buffers free
            for (int idx = threadIdx.x; idx < (cnt << lgNf); idx += NT) {
                const int q = idx / cnt, f = idx - q * cnt;
                const int i = (q < (Nf >> 1) ? q : q - Nf) + M;
                fa[(f << lgNf) + q] =
                    (i >= 0 && i < L) ? R[(size_t)i * H + v0 + f] : make_float2(0.f, 0.f);
            }
            const float2 *X = fft_batch<NT>(fa, fb, lgNf, cnt, twf, false);
            for (int idx = threadIdx.x; idx < (cnt << lgNf); idx += NT) {
                const int u = idx / cnt, f = idx - u * cnt;
                B[(size_t)u * H + v0 + f] = X[(f << lgNf) + u];
            }
        }
        __syncthreads();  // B written
        const bool isbad = sbad != 0;
        float *out = pmf + g * (int64_t)n * L;
        // 3. slices theta_m, m < n/2, two per inverse transform
        for (int m0 = 0; m0 < (n >> 1); m0 += 2 * GS) {
            const int ns = min(2 * GS, (n >> 1) - m0);  // even: n is a multiple of 8
            for (int idx = threadIdx.x; idx < ns * (M + 1); idx += NT) {
                const int sl = idx / (M + 1), k = idx - sl * (M + 1);
                const double2 d = d64[m0 + sl];
                Y[idx] = slice_point(B, Nf, H, L, d.x, d.y, k, S.beta);
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < ((ns >> 1) << lgL); idx += NT) {
                const int f = idx >> lgL, t = idx & (L - 1);
                const int k = t < M ? t : t - L;
                const float2 *Y1 = Y + (2 * f) * (M + 1), *Y2 = Y1 + (M + 1);
                float2 c1 = k >= 0 ? Y1[k] : Y1[-k], c2 = k >= 0 ? Y2[k] : Y2[-k];
                if (k < 0) {  // the coefficients of a real projection are Hermitian
                    c1.y = -c1.y;
                    c2.y = -c2.y;
                }
                float2 z1 = cmul(c1, shf[t]), z2 = cmul(c2, shf[t]);
                if (k == 0 || k == -M) {  // self-paired frequencies: real part
                    z1.y = 0.f;
                    z2.y = 0.f;
                }
                fa[idx] = make_float2(z1.x - z2.y, z1.y + z2.x);  // z1 + i z2
            }
            const float2 *X = fft_batch<NT>(fa, fb, lgL, ns >> 1, twl, true);
            for (int idx = threadIdx.x; idx < ((ns >> 1) << lgL); idx += NT) {
                const int f = idx >> lgL, b = idx & (L - 1);
                const float2 z = X[idx];
                const int m1 = m0 + 2 * f, m2 = m1 + 1;
                const float qnan = __int_as_float(0x7fc00000);
                const float p1 = isbad ? qnan : fmaxf(0.5f * h * z.x, 0.f);
                const float p2 = isbad ? qnan : fmaxf(0.5f * h * z.y, 0.f);
                out[(int64_t)m1 * L + b] = p1;
                out[(int64_t)(m1 + (n >> 1)) * L + (L - 1 - b)] = p1;
                out[(int64_t)m2 * L + b] = p2;
                out[(int64_t)(m2 + (n >> 1)) * L + (L - 1 - b)] = p2;
            }
            __syncthreads();  // Y and the work buffers are rewritten next round
        }
    }
}

}  // namespace

size_t fourier_lds_bytes(int L, int Nf) {
    const int M = L / 2;
    return sizeof(float2) * (2 * kFftFloats2 + (2 * kFftFloats2 / L) * (M + 1) + Nf / 2 + L / 2 + L) +
           sizeof(float) * L;
}

size_t fourier_slot_bytes(int L, int Nf) { return sizeof(float2) * (size_t)(L + Nf) * (Nf / 2 + 1); }

hipError_t launch_fourier(const float *img, int64_t N, const FourierShape &S, const FourierTabs &T,
                          const AngleTable &t, void *scratch, int slots, float *pmf,
                          hipStream_t s) {
    if (N <= 0) return hipSuccess;
    constexpr int NT = 256;
    const size_t lds = fourier_lds_bytes(S.L, S.Nf);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_fourier<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)attr;
    const int grid = (int)(N < slots ? N : slots);
    hipLaunchKernelGGL((k_fourier<NT>), dim3(grid), dim3(NT), lds, s, img, N, S, T, t.d64,
                       (float2 *)scratch, pmf);
    return hipGetLastError();
}

}  // namespace sw
