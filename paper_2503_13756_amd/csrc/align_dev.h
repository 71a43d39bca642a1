// Angle spectra and pairwise alignment of quantile tables.
//
// Sec. 2.3 (fast computation over rotations): a rotation of the image is a
// cyclic shift of the columns of its quantile table, and the cross term
// sum_{j,k} U[j][k] V[j][k+l] of the squared distance is, for every lag l at
// once, a cross-correlation along the angle axis, done by FFT row by row and
// summed over rows.  Summing over rows before the inverse transform leaves one
// length-n inverse transform per pair:
//   S(w) = sum_j conj(U^_j(w)) V^_j(w),
//   C(l) = (1/n) sum_w S(w) e^{2 pi i w l / n}.
// The translation at every lag is the least-squares shift of the quantile
// functions, which by the translation equivariance of SW2 (Thm 3.2 and its
// proof) reduces to the first angular moment of the column means:
//   b(l) = a_U - e^{i theta_l} a_V,  s*(l) = 2 b(l),  D*(l) = D0(l) - 2|b(l)|^2.
//
// FFTs: two real table rows are packed into one complex row and transformed
// by a Stockham FFT in LDS (radix 4, 3, 2, ping-pong between two buffers;
// twiddles from the angle table, which equals e^{-2 pi i m / n}); the two
// real spectra are separated from the packed one by conjugate symmetry.
#pragma once
#include <type_traits>
#include "fft_dev.h"

namespace sw {

// Complex elements of one LDS FFT chunk (8 KiB, two buffers).  The per-pair
// alignment is latency bound: small chunks keep its LDS near 22 KiB at
// n = 256, so that seven blocks fit on a compute unit instead of two.
constexpr int kFftElems = 1024;

// bfloat16 round-to-nearest-even of two floats, returned as floats: one
// v_cvt_pk_bf16_f32 for the pair (round to nearest even; equal to the bit
// formula u + 0x7fff + ((u >> 16) & 1), truncated, on every non-NaN float),
// then the halves shifted back
__device__ __forceinline__ float2 bf16r2(float2 v) {
    const __bf16 a = (__bf16)v.x, b = (__bf16)v.y;
    return make_float2((float)a, (float)b);
}

// Load complex rows p0 .. p0+rows-1 of a [Q][n] real table: row p packs table
// rows 2p (real part) and 2p+1 (imaginary part).
template <int NT>
__device__ void load_packed(float2 *Z, const float *__restrict__ T, int n, int p0, int rows) {
    for (int idx = threadIdx.x; idx < rows * n; idx += NT) {
        const int pl = idx / n, k = idx - pl * n;
        const int j = 2 * (p0 + pl);
        Z[idx] = make_float2(T[(int64_t)j * n + k], T[(int64_t)(j + 1) * n + k]);
    }
}

// Separate the spectra of the two real rows packed in Z row pl at frequency w.
__device__ __forceinline__ void unpack(const float2 *Z, int pl, int n, int w, float2 &xe,
                                       float2 &xo) {
    const float2 zw = Z[pl * n + w];
    const float2 zc = Z[pl * n + (w == 0 ? 0 : n - w)];
    // xe = (zw + conj(zc)) / 2 ; xo = (zw - conj(zc)) / (2i)
    xe = make_float2(0.5f * (zw.x + zc.x), 0.5f * (zw.y - zc.y));
    const float dx = zw.x - zc.x, dy = zw.y + zc.y;
    xo = make_float2(0.5f * dy, -0.5f * dx);
}

__device__ __forceinline__ int fft_chunk_rows(int n, int Q) {
    const int c = kFftElems / n;
    return c < Q / 2 ? c : Q / 2;
}

// -------------------------------------------------------------- alignment
__device__ __forceinline__ void argmin_merge(double &v, int &i, double v2, int i2) {
    if (v2 < v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

template <int NT>
__device__ int block_argmin(const double *D, int n, double *rv, int *ri) {
    double v = __builtin_inf();
    int i = 0x7fffffff;
    for (int l = threadIdx.x; l < n; l += NT) argmin_merge(v, i, D[l], l);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double v2 = __shfl_xor(v, off, 64);
        const int i2 = __shfl_xor(i, off, 64);
        argmin_merge(v, i, v2, i2);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        rv[wave] = v;
        ri[wave] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NT / 64; ++w) argmin_merge(v, i, rv[w], ri[w]);
        ri[0] = i;
    }
    __syncthreads();
    const int r = ri[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ float block_sum(float v, float *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        red[0] = s;
    }
    __syncthreads();
    s = red[0];
    __syncthreads();
    return s;
}

// b(l) = a_U - e^{i theta_l} a_V
__device__ __forceinline__ double2 trans_moment(const double *au, const double *av, double2 d) {
    const double c = d.x, s = -d.y;
    return make_double2(au[2] - (c * av[2] - s * av[3]), au[3] - (s * av[2] + c * av[3]));
}

// Angle spectra of one [Q][n] table into spec[w][j] (float2, or packed bf16
// complex when bf16 != 0).  lds: n + 2 kFftElems float2.
template <int NT>
__device__ void spectrum_block(const float *__restrict__ T, int n, int Q, void *spec, int bf16,
                               const float2 *__restrict__ tw32, float2 *lds2) {
    const int Wn = n / 2 + 1;
    float2 *tw = lds2;
    float2 *Z0 = lds2 + n;
    float2 *Z1 = Z0 + kFftElems;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) tw[i] = tw32[i];
    const int CH = fft_chunk_rows(n, Q);
    for (int p0 = 0; p0 < Q / 2; p0 += CH) {
        const int rows = min(CH, Q / 2 - p0);
        __syncthreads();
        load_packed<NT>(Z0, T, n, p0, rows);
        __syncthreads();
        const float2 *Z = fft_rows<NT>(Z0, Z1, rows, n, tw);
        for (int idx = threadIdx.x; idx < rows * Wn; idx += NT) {
            const int w = idx / rows, pl = idx - w * rows;
            float2 xe, xo;
            unpack(Z, pl, n, w, xe, xo);
            const int64_t o = (int64_t)w * Q + 2 * (p0 + pl);
            if (bf16) {
                uint32_t *sp = (uint32_t *)spec;
                const float2 e = bf16r2(xe), d = bf16r2(xo);
                sp[o] = (__float_as_uint(e.x) >> 16) | (__float_as_uint(e.y) & 0xffff0000u);
                sp[o + 1] = (__float_as_uint(d.x) >> 16) | (__float_as_uint(d.y) & 0xffff0000u);
            } else {
                float2 *sp = (float2 *)spec;
                sp[o] = xe;
                sp[o + 1] = xo;
            }
        }
    }
    __syncthreads();
}

// Alignment of one table pair by one block: spectra of V, spectral dot with
// the reference spectrum Uh, inverse transform over the lags, translation
// correction, top-k, FP32 rescore; writes *res (and curve[0..n) if given).
// lds: n + 2 kFftElems + Wn G float2 followed by n doubles.
struct PairJob {
    const float *U, *V;       // [Q][n] tables
    const double *au, *av;    // aux of both
    const float2 *Uh;         // [Wn][Q] FP32 spectrum of U
    Result *res;
    float *curve;             // nullable, [n]
    int status;               // precomputed status (0 = compute)
};

template <int NT>
__device__ void align_pair_block(const PairJob &job, Geo g, int mode, int bf16, int top_k,
                                 const float2 *__restrict__ tw32, const double2 *__restrict__ tw64,
                                 float2 *lds2) {
    __shared__ double rv[NT / 64];
    __shared__ int ri[NT / 64];
    __shared__ float rf[NT / 64];
    __shared__ int cand[kMaxTopK];
    const int n = g.n, Q = g.Q, Wn = n / 2 + 1;
    const int G = Wn >= NT ? 1 : NT / Wn;
    float2 *tw = lds2;
    float2 *Z0 = tw + n;
    float2 *Z1 = Z0 + kFftElems;
    float2 *Sacc = Z1 + kFftElems;
    double *D = (double *)(Sacc + Wn * G);
    Result *res = job.res;
    __syncthreads();  // the previous job of this block may still read LDS
    if (job.status) {
        if (threadIdx.x == 0) {
            res->rot_index = 0;
            res->theta_rad = 0.f;
            res->shift_px[0] = res->shift_px[1] = 0.f;
            res->sw2sq = __int_as_float(0x7fc00000);
            res->status = job.status;
        }
        if (job.curve)
            for (int l = threadIdx.x; l < n; l += NT) job.curve[l] = __int_as_float(0x7fc00000);
        return;
    }
    const float *U = job.U, *V = job.V;
    const double *au = job.au, *av = job.av;
    const float2 *Uh = job.Uh;

    for (int i = threadIdx.x; i < n; i += NT) tw[i] = tw32[i];
    for (int i = threadIdx.x; i < Wn * G; i += NT) Sacc[i] = make_float2(0.f, 0.f);

    // --- spectra of V and the spectral dot with conj(U^)
    const int CH = fft_chunk_rows(n, Q);
    for (int p0 = 0; p0 < Q / 2; p0 += CH) {
        const int rows = min(CH, Q / 2 - p0);
        __syncthreads();
        load_packed<NT>(Z0, V, n, p0, rows);
        __syncthreads();
        const float2 *Z = fft_rows<NT>(Z0, Z1, rows, n, tw);
        // the rounding to bf16 as a compile-time choice: as a run-time flag
        // the compiler rounds on both paths and selects
        auto dot = [&](auto round) {
            for (int it = threadIdx.x; it < Wn * G; it += NT) {
                const int w = it / G, gg = it - w * G;
                float2 s = Sacc[it];
                for (int pl = gg; pl < rows; pl += G) {
                    float2 xe, xo;
                    unpack(Z, pl, n, w, xe, xo);
                    const float4 uu = *(const float4 *)(Uh + (int64_t)w * Q + 2 * (p0 + pl));
                    float2 ue = make_float2(uu.x, uu.y), uo = make_float2(uu.z, uu.w);
                    if constexpr (decltype(round)::value) {
                        xe = bf16r2(xe);
                        xo = bf16r2(xo);
                        ue = bf16r2(ue);
                        uo = bf16r2(uo);
                    }
                    // conj(ue) * xe + conj(uo) * xo
                    s.x += ue.x * xe.x + ue.y * xe.y + uo.x * xo.x + uo.y * xo.y;
                    s.y += ue.x * xe.y - ue.y * xe.x + uo.x * xo.y - uo.y * xo.x;
                }
                Sacc[it] = s;
            }
        };
        if (bf16)
            dot(std::true_type{});
        else
            dot(std::false_type{});
    }
    __syncthreads();
    float2 *S = Z0;  // reuse
    for (int w = threadIdx.x; w < Wn; w += NT) {
        float2 s = make_float2(0.f, 0.f);
        for (int gg = 0; gg < G; ++gg) {
            s.x += Sacc[w * G + gg].x;
            s.y += Sacc[w * G + gg].y;
        }
        S[w] = s;
    }
    __syncthreads();

    // --- inverse transform over w, translation correction, objective per lag
    const double nq = (double)n * (double)Q;
    for (int l = threadIdx.x; l < n; l += NT) {
        float acc = S[0].x + ((l & 1) ? -S[n / 2].x : S[n / 2].x);
        float part = 0.f;
        int m = l;
        for (int w = 1; w < n / 2; ++w) {
            const float2 t = tw[m];
            part += S[w].x * t.x + S[w].y * t.y;  // Re(S e^{+2 pi i w l / n})
            m += l;
            if (m >= n) m -= n;
        }
        const double Cl = ((double)acc + 2.0 * (double)part) / (double)n;
        double d = (au[1] + av[1] - 2.0 * Cl) / nq;
        if (mode == 0) {
            const double2 b = trans_moment(au, av, tw64[l]);
            d -= 2.0 * (b.x * b.x + b.y * b.y);
        }
        D[l] = d;
        if (job.curve) job.curve[l] = (float)d;
    }
    __syncthreads();

    // --- top-K lags
    const int K = top_k;
    for (int c = 0; c < K; ++c) {
        const int l = block_argmin<NT>(D, n, rv, ri);
        if (threadIdx.x == 0) {
            cand[c] = l;
            D[l] = __builtin_inf();
        }
        __syncthreads();
    }

    // --- FP32 rescore of the candidates: direct residual sum
    float sx[kMaxTopK], sy[kMaxTopK], part[kMaxTopK];
    int lc[kMaxTopK];
#pragma unroll
    for (int c = 0; c < kMaxTopK; ++c) {
        lc[c] = c < K ? cand[c] : 0;
        double2 b = make_double2(0.0, 0.0);
        if (mode == 0 && c < K) b = trans_moment(au, av, tw64[lc[c]]);
        sx[c] = (float)(2.0 * b.x);
        sy[c] = (float)(2.0 * b.y);
        part[c] = 0.f;
    }
    // rows of V pass through LDS (the FFT buffers, free by now): every element
    // is read once from memory and K times from LDS
    float *Vs = (float *)Z0;
    const int RS = 4 * kFftElems / n;
    for (int j0 = 0; j0 < Q; j0 += RS) {
        const int cnt = min(RS, Q - j0) * n;
        const float *Vg = V + (int64_t)j0 * n;
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt; idx += NT) Vs[idx] = Vg[idx];
        __syncthreads();
        const float *Ug = U + (int64_t)j0 * n;
        for (int idx = threadIdx.x; idx < cnt; idx += NT) {
            const int jl = idx / n, k = idx - jl * n;
            const float u = Ug[idx];
            const float2 dk = tw[k];
            const float *vrow = Vs + jl * n;
#pragma unroll
            for (int c = 0; c < kMaxTopK; ++c) {
                if (c < K) {
                    int kk = k + lc[c];
                    if (kk >= n) kk -= n;
                    const float e = u - vrow[kk] - (sx[c] * dk.x + sy[c] * dk.y);
                    part[c] += e * e;
                }
            }
        }
    }
    int best_l = 0;
    float best = 0.f, bsx = 0.f, bsy = 0.f;
    for (int c = 0; c < K; ++c) {
        const float v = block_sum<NT>(part[c], rf) / (float)nq;
        if (c == 0 || v < best || (v == best && lc[c] < best_l)) {
            best = v;
            best_l = lc[c];
            bsx = sx[c];
            bsy = sy[c];
        }
    }
    if (threadIdx.x == 0) {
        const float L = (float)g.L;
        res->rot_index = best_l;
        res->theta_rad = (float)(6.283185307179586 * (double)best_l / (double)n);
        res->shift_px[0] = bsx * 0.5f * L;
        res->shift_px[1] = bsy * 0.5f * L;
        res->sw2sq = best;
        res->status = 0;
    }
}

}  // namespace sw
