// Fourier-slice projector (Sec. 2.2: the 1-D Fourier transform of the line
// projection at angle theta is the central slice of the image's 2-D Fourier
// transform; Sec. 2.3 computes the slices with a NUFFT and returns to the
// detector with a 1-D inverse DFT).  The discretisation is that of the
// appendix's fixed-angle error theorem with NUFFT precision: slice
// frequencies k pi, k = -M .. M-1 (L = 2M), and the trigonometric polynomial
// with coefficients yhat_k / 2 sampled at the detector bin centres.
//
// One 512-thread block per image slot of a persistent grid (as many slots as
// fit on the CUs at once); per image:
//  1. rows: the pixel masses (positive part inside the disk, exactly as for
//     the line sum) divided by the kernel's Fourier transform at their
//     centred index, zero-padded to Nf = 2L and transformed along x; two
//     real rows share one complex FFT.  The half spectrum v <= Nf/2 goes to
//     the slot's scratch (R).
//  2. columns: the same transform along y for every v <= Nf/2 (B, the
//     oversampled spectrum; the other half is its conjugate mirror).
//  3. slices: every slice point k pi d_theta (theta in [0, pi), k = 0..M, or
//     every given angle) is
//     interpolated from B with a separable exponential-of-semicircle kernel
//     of width kW, phase-shifted to the pixel centres and multiplied by the
//     transform of one pixel cell; the coefficients of two slices are packed
//     into one complex L-point inverse FFT (both results are real), scaled by
//     h/2, clipped at zero and written with their theta + pi mirror.
// The FFTs are Stockham transforms in LDS over a batch of sequences: for L a
// power of two radix 4 with one radix-2 step for odd powers, with shift and
// mask indexing; for other L (factors 2 and 3) the mixed-radix transforms of
// fft_dev.h, the inverse as conj(FFT(conj x)).
#include "fft_dev.h"
#include "fourier_internal.h"

namespace sw {

namespace {

constexpr int kFftFloats2 = 2048;  // float2 per FFT work buffer

__device__ __forceinline__ bool in_disk_f(int L, int i, int j) {
    const int a = 2 * j - L + 1, b = 2 * i - L + 1, r = L - 2;
    return a * a + b * b <= r * r;
}

// One Stockham step of radix R over cnt transforms of length 2^lg: element
// j + r 2^lg / R of each transform, twiddled by exp(-+2 pi i r (j mod Ns) /
// (Ns R)), goes through an R-point DFT to position (j / Ns) Ns R + (j mod Ns)
// + r Ns of the output.
template <int NT, int R>
__device__ __forceinline__ void fft_step(const float2 *a, float2 *b, int lg, int lgNs, int cnt,
                                         const float2 *tw, bool inv) {
    constexpr int lgR = R == 4 ? 2 : 1;
    const int nq = 1 << (lg - lgR), Ns = 1 << lgNs;
    for (int idx = threadIdx.x; idx < cnt * nq; idx += NT) {
        const int f = idx >> (lg - lgR), j = idx & (nq - 1);
        const float2 *src = a + (f << lg);
        float2 *dst = b + (f << lg);
        const int jm = j & (Ns - 1);
        const int o = ((j - jm) << lgR) + jm;
        // twiddle index of r = 1: jm N / (Ns R)
        const int t1 = jm << (lg - lgNs - lgR);
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = src[j + r * nq];
            if (r > 0) {
                float2 w = tw[r * t1];
                if (inv) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
        }
        if (R == 2) {
            dst[o] = make_float2(v[0].x + v[1].x, v[0].y + v[1].y);
            dst[o + Ns] = make_float2(v[0].x - v[1].x, v[0].y - v[1].y);
        } else {
            const float2 a0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
            const float2 a1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
            const float2 a2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
            // (v1 - v3) times -i (forward) or +i (inverse)
            const float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
            const float2 a3 = inv ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
            dst[o] = make_float2(a0.x + a2.x, a0.y + a2.y);
            dst[o + Ns] = make_float2(a1.x + a3.x, a1.y + a3.y);
            dst[o + 2 * Ns] = make_float2(a0.x - a2.x, a0.y - a2.y);
            dst[o + 3 * Ns] = make_float2(a1.x - a3.x, a1.y - a3.y);
        }
    }
}

// cnt transforms of length 2^lg held at a[f << lg .. ]; b is a work buffer of
// the same size.  tw[k] = exp(-2 pi i k / 2^lg) for k < 2^lg; inv selects the
// conjugate twiddles (exp(+2 pi i ...)).  Stockham steps of radix 4 (one of
// radix 2 first when lg is odd).  Inputs must be visible to the whole block
// on entry; returns the buffer holding the (naturally ordered) result,
// visible to the whole block.
template <int NT>
__device__ float2 *fft_batch(float2 *a, float2 *b, int lg, int cnt, const float2 *tw, bool inv) {
    int lgNs = 0;
    if (lg & 1) {
        __syncthreads();
        fft_step<NT, 2>(a, b, lg, 0, cnt, tw, inv);
        float2 *x = a;
        a = b;
        b = x;
        lgNs = 1;
    }
    for (; lgNs < lg; lgNs += 2) {
        __syncthreads();
        fft_step<NT, 4>(a, b, lg, lgNs, cnt, tw, inv);
        float2 *x = a;
        a = b;
        b = x;
    }
    __syncthreads();
    return a;
}

// Slice value yhat at one slice point from the oversampled spectrum, stored
// with kFourierPad conjugate-mirrored columns on both sides (row length Hx,
// column v at v + kFourierPad), so that every tap is a plain load.  The
// target entry (host-built per geometry, float4 x 5): (u0, v0 | conj << 16)
// as ints and the complex factor (pixel-centre phase times the cell
// transform); the kW x-weights; the kW y-weights.  Taps are rows
// (u0 + a) mod Nf, columns v0 - kFourierPad + c; with conj the kernel was
// evaluated at the mirrored point and the sum is conjugated.
template <bool POW2>
__device__ __forceinline__ float2 slice_point(const float2 *__restrict__ B, int Nf, int Hx,
                                              const float4 *__restrict__ e) {
    const float4 e0 = e[0], e1 = e[1], e2 = e[2], e3 = e[3], e4 = e[4];
    const int u0 = __float_as_int(e0.x), vw = __float_as_int(e0.y);
    const float wx[kFourierW] = {e1.x, e1.y, e1.z, e1.w, e2.x, e2.y, e2.z};
    const float wy[kFourierW] = {e3.x, e3.y, e3.z, e3.w, e4.x, e4.y, e4.z};
    const float2 *col = B + (vw & 0xffff);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < kFourierW; ++a) {
        int u;  // (u0 + a) mod Nf: u0 < Nf, a < kFourierW <= Nf
        if constexpr (POW2) u = (u0 + a) & (Nf - 1);
        else u = u0 + a < Nf ? u0 + a : u0 + a - Nf;
        const float2 *row = col + u * Hx;
        float2 ra = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < kFourierW; ++c) {
            const float2 bv = row[c];
            ra.x = fmaf(wx[c], bv.x, ra.x);
            ra.y = fmaf(wx[c], bv.y, ra.y);
        }
        acc.x = fmaf(wy[a], ra.x, acc.x);
        acc.y = fmaf(wy[a], ra.y, acc.y);
    }
    if (vw >> 16) acc.y = -acc.y;
    return cmul(acc, make_float2(e0.z, e0.w));
}

// Multiples and quotients by a transform length: shifts for powers of two,
// else plain arithmetic.
template <bool POW2>
struct Len {
    int n, lg;
    __device__ __forceinline__ int mul(int x) const {
        if constexpr (POW2) return x << lg;
        else return x * n;
    }
    __device__ __forceinline__ int div(int x) const {
        if constexpr (POW2) return x >> lg;
        else return x / n;
    }
};

template <int NT, bool POW2>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fourier(const float *__restrict__ img, int64_t N,
                                                FourierShape S, FourierTabs T,
                                                float2 *__restrict__ scratch, float *__restrict__ pmf) {
    extern __shared__ __align__(16) float2 lds2[];
    __shared__ int sbad;
    const int L = S.L, M = L >> 1, n = S.n, Nf = S.Nf, H = S.H, lgNf = S.lgNf, lgL = S.lgL;
    const int Hx = H + 2 * kFourierPad - 1;
    const float h = 2.f / (float)L;
    float2 *fa = lds2, *fb = lds2 + kFftFloats2;
    float2 *Y = fb + kFftFloats2;                      // [slices][M + 1]
    float2 *twf = Y + (2 * kFftFloats2 / L) * (M + 1);  // [Nf]
    float2 *twl = twf + Nf;                             // [L]
    float2 *shf = twl + L;                              // [L]
    float *corr = (float *)(shf + L);                   // [L]
    for (int t = threadIdx.x; t < Nf; t += NT) twf[t] = T.twf[t];
    for (int t = threadIdx.x; t < L; t += NT) twl[t] = T.twl[t];
    for (int t = threadIdx.x; t < L; t += NT) {
        shf[t] = T.shift[t];
        corr[t] = T.corr[t];
    }
    float2 *R = scratch + (size_t)blockIdx.x * fourier_slot_elems(L, Nf);  // [L][H]
    float2 *B = R + (size_t)L * H;  // [Nf][Hx], column v at v + kFourierPad
    const Len<POW2> LF{Nf, lgNf}, LH{Nf >> 1, lgNf - 1}, LL{L, lgL};
    const int GR = kFftFloats2 / Nf;  // transforms of length Nf per round
    const int GS = kFftFloats2 / L;   // transforms of length L per round (two slices each)
    // forward transforms of cnt sequences of length len (twiddles tw); the
    // input must be complete in LDS, the result is visible to the block
    auto fft = [&](float2 *a, float2 *b, int cnt, int len, int lg, const float2 *tw) -> float2 * {
        if constexpr (POW2) {
            return fft_batch<NT>(a, b, lg, cnt, tw, false);
        } else {
            __syncthreads();
            return fft_rows<NT>(a, b, cnt, len, tw);
        }
    };
    for (int64_t g = blockIdx.x; g < N; g += gridDim.x) {
        const float *F = img + g * (int64_t)L * L;
        __syncthreads();  // previous image done with sbad and the buffers
        if (threadIdx.x == 0) sbad = 0;
        int bad = 0;
        // 1. rows, two per transform
        for (int p0 = 0; p0 < M; p0 += GR) {
            const int cnt = min(GR, M - p0);
            __syncthreads();
            for (int idx = threadIdx.x; idx < LF.mul(cnt); idx += NT) {
                const int f = LF.div(idx), q = idx - LF.mul(f);
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
            const float2 *X = fft(fa, fb, cnt, Nf, lgNf, twf);
            auto unpack = [&](int f, int v) {
                const float2 zv = X[LF.mul(f) + v], zc = X[LF.mul(f) + (v == 0 ? 0 : Nf - v)];
                const int i = 2 * (p0 + f);
                // Z = X_i + i X_{i+1}: X_i[v] = (Z[v] + conj Z[-v]) / 2,
                // X_{i+1}[v] = (Z[v] - conj Z[-v]) / (2 i)
                R[(size_t)i * H + v] = make_float2(0.5f * (zv.x + zc.x), 0.5f * (zv.y - zc.y));
                R[(size_t)(i + 1) * H + v] = make_float2(0.5f * (zv.y + zc.y), -0.5f * (zv.x - zc.x));
            };
            for (int idx = threadIdx.x; idx < LH.mul(cnt); idx += NT) {
                const int f = LH.div(idx);
                unpack(f, idx - LH.mul(f));
            }
            for (int f = threadIdx.x; f < cnt; f += NT) unpack(f, Nf >> 1);  // v = Nf/2
        }
        if (bad) sbad = 1;
        // 2. columns
        for (int v0 = 0; v0 < H; v0 += GR) {
            const int cnt = min(GR, H - v0);
            __syncthreads();  // R written; work buffers free
            // element idx = q cnt + f (f fastest: neighbouring threads take
            // neighbouring columns); cnt is a power of two except for L <= 16
            const int lgc = 31 - __builtin_clz(cnt);
            const bool p2 = (1 << lgc) == cnt;
            auto load = [&](int q, int f) {
                const int i = (q < (Nf >> 1) ? q : q - Nf) + M;
                fa[LF.mul(f) + q] =
                    (i >= 0 && i < L) ? R[(size_t)i * H + v0 + f] : make_float2(0.f, 0.f);
            };
            if (p2) {
                for (int idx = threadIdx.x; idx < LF.mul(cnt); idx += NT)
                    load(idx >> lgc, idx & (cnt - 1));
            } else {
                for (int idx = threadIdx.x; idx < LF.mul(cnt); idx += NT)
                    load(idx / cnt, idx % cnt);
            }
            const float2 *X = fft(fa, fb, cnt, Nf, lgNf, twf);
            auto store = [&](int u, int f) { B[(size_t)u * Hx + kFourierPad + v0 + f] = X[LF.mul(f) + u]; };
            if (p2) {
                for (int idx = threadIdx.x; idx < LF.mul(cnt); idx += NT)
                    store(idx >> lgc, idx & (cnt - 1));
            } else {
                for (int idx = threadIdx.x; idx < LF.mul(cnt); idx += NT) store(idx / cnt, idx % cnt);
            }
        }
        __syncthreads();  // B written
        // mirrored pad columns: B[u][v] = conj B[-u][-v] for v < 0 and for
        // v > Nf/2 (there as B[-u][Nf - v])
        for (int idx = threadIdx.x; idx < Nf * (2 * kFourierPad - 1); idx += NT) {
            const int u = idx / (2 * kFourierPad - 1), c = idx - u * (2 * kFourierPad - 1);
            const int v = c < kFourierPad ? c - kFourierPad : (Nf >> 1) + 1 + (c - kFourierPad);
            const int vs = v < 0 ? -v : Nf - v;
            float2 z = B[(size_t)(u == 0 ? 0 : Nf - u) * Hx + kFourierPad + vs];
            z.y = -z.y;
            B[(size_t)u * Hx + kFourierPad + v] = z;
        }
        __syncthreads();
        const bool isbad = sbad != 0;
        float *out = pmf + g * (int64_t)n * L;
        // 3. slices theta_m, m < n/2, two per inverse transform
        // slices m < nsl: nsl = n/2 with their theta + pi mirrors, or all n
        // (slices at explicit angles)
        const int nsl = S.mirror ? (n >> 1) : n;
        for (int m0 = 0; m0 < nsl; m0 += 2 * GS) {
            const int ns = min(2 * GS, nsl - m0);  // even: n is a multiple of 8
            for (int idx = threadIdx.x; idx < ns * (M + 1); idx += NT)
                Y[idx] = slice_point<POW2>(B, Nf, Hx, T.targets + 5 * ((size_t)m0 * (M + 1) + idx));
            __syncthreads();
            for (int idx = threadIdx.x; idx < LL.mul(ns >> 1); idx += NT) {
                const int f = LL.div(idx), t = idx - LL.mul(f);
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
                float2 zz = make_float2(z1.x - z2.y, z1.y + z2.x);  // z1 + i z2
                if constexpr (!POW2) zz.y = -zz.y;  // inverse as conj(FFT(conj))
                fa[idx] = zz;
            }
            const float2 *X;
            if constexpr (POW2) X = fft_batch<NT>(fa, fb, lgL, ns >> 1, twl, true);
            else X = fft(fa, fb, ns >> 1, L, lgL, twl);
            for (int idx = threadIdx.x; idx < LL.mul(ns >> 1); idx += NT) {
                const int f = LL.div(idx), b = idx - LL.mul(f);
                float2 z = X[idx];
                if constexpr (!POW2) z.y = -z.y;
                const int m1 = m0 + 2 * f, m2 = m1 + 1;
                const float qnan = __int_as_float(0x7fc00000);
                const float p1 = isbad ? qnan : fmaxf(0.5f * h * z.x, 0.f);
                const float p2 = isbad ? qnan : fmaxf(0.5f * h * z.y, 0.f);
                out[(int64_t)m1 * L + b] = p1;
                out[(int64_t)m2 * L + b] = p2;
                if (S.mirror) {
                    out[(int64_t)(m1 + (n >> 1)) * L + (L - 1 - b)] = p1;
                    out[(int64_t)(m2 + (n >> 1)) * L + (L - 1 - b)] = p2;
                }
            }
            __syncthreads();  // Y and the work buffers are rewritten next round
        }
    }
}

}  // namespace

size_t fourier_lds_bytes(int L, int Nf) {
    const int M = L / 2;
    return sizeof(float2) * (2 * kFftFloats2 + (2 * kFftFloats2 / L) * (M + 1) + Nf + L + L) +
           sizeof(float) * L;
}

size_t fourier_slot_bytes(int L, int Nf) { return sizeof(float2) * fourier_slot_elems(L, Nf); }

constexpr int kFourierNT = 512;

static void fourier_attr() {
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)k_fourier<kFourierNT, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    static const hipError_t attr2 =
        hipFuncSetAttribute((const void *)k_fourier<kFourierNT, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)attr;
    (void)attr2;
}

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int fourier_blocks_per_cu(int L, int Nf) {
    fourier_attr();
    int nb = 0;
    const hipError_t e =
        is_pow2(L) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fourier<kFourierNT, true>,
                                                                  kFourierNT, fourier_lds_bytes(L, Nf))
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fourier<kFourierNT, false>,
                                                                  kFourierNT, fourier_lds_bytes(L, Nf));
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_fourier(const float *img, int64_t N, const FourierShape &S, const FourierTabs &T,
                          void *scratch, int slots, float *pmf, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    constexpr int NT = kFourierNT;
    const size_t lds = fourier_lds_bytes(S.L, S.Nf);
    fourier_attr();
    const int grid = (int)(N < slots ? N : slots);
    if (is_pow2(S.L))
        hipLaunchKernelGGL((k_fourier<NT, true>), dim3(grid), dim3(NT), lds, s, img, N, S, T,
                           (float2 *)scratch, pmf);
    else
        hipLaunchKernelGGL((k_fourier<NT, false>), dim3(grid), dim3(NT), lds, s, img, N, S, T,
                           (float2 *)scratch, pmf);
    return hipGetLastError();
}

}  // namespace sw
