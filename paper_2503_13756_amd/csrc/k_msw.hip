// Max-sliced alignment (extended alignment results: the max-sliced W2 over
// the equispaced slices, the norm of U - V taken over columns), rotation only:
//   M(l) = max_k (1/Q) sum_j (U[j][k] - V[j][(k+l) mod n])^2,  l* = argmin M.
// The column pairing of every lag at once is the n x n product
// C[k][k'] = sum_j U[j][k] V[j][k'] = (U^T V)[k][k'], run on the matrix cores
// in FP32 (v_mfma_f32_16x16x4f32): the lag-l residual of column k is
// |u_k|^2 + |v_{k+l}|^2 - 2 C[k][k+l], and the max over k per lag is an LDS
// atomic max over the diagonals of C.  The top_k lags of that FP32 estimate
// are then rescored as direct residual sums (no cancellation), and the
// smallest rescored value wins (ties to the smaller lag).
//
// One 4-wave block per pair, n a multiple of 16 up to 128.  Wave w owns the
// row blocks a = w, w + 4 (those below n / 16) of the 16 x 16 tiles of C and
// all column blocks; V streams through LDS in chunks
// of 64 rows (row stride n + 16 floats, so the four rows of a B fragment fall
// in distinct banks), U comes straight from global memory (the reference
// tables are L2-resident).
#include "sw_internal.h"

namespace sw {

typedef float f32x4m __attribute__((ext_vector_type(4)));

template <int NN>
__global__ __launch_bounds__(256) void k_align_msw(PairArgs a, Geo g) {
    static_assert(NN % 16 == 0 && NN <= 128, "n a multiple of 16 up to 128");
    constexpr int NB = NN / 16, RA = (NB + 3) / 4, KC = 64, VS = NN + 16;
    __shared__ float vs[KC * VS];
    __shared__ float uu[NN], vv[NN];
    __shared__ unsigned Dbits[NN];
    __shared__ float colred[256];
    __shared__ int cand[kMaxTopK];
    __shared__ float cval[kMaxTopK];
    const int Q = g.Q;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t pi = blockIdx.x;
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (pi >= P) return;
    const int64_t r = a.pairs ? a.pairs[2 * pi] : pi / a.n_img;
    const int64_t gi = a.pairs ? a.pairs[2 * pi + 1] : pi % a.n_img;
    const bool in_range = r >= 0 && r < a.n_ref && gi >= 0 && gi < a.n_img;
    Result *res = a.out + pi;
    float *curve = a.curve ? a.curve + pi * NN : nullptr;
    int status = 0;
    const double *au = a.ref_aux + 4 * (in_range ? r : 0), *av = a.img_aux + 4 * (in_range ? gi : 0);
    if (!in_range) status = 3;  // bad pair index
    else if (isnan(au[0]) || isnan(av[0])) status = 2;
    else if (!(au[0] > 0.0) || !(av[0] > 0.0)) status = 1;
    if (status) {
        if (t == 0) {
            res->rot_index = 0;
            res->theta_rad = 0.f;
            res->shift_px[0] = res->shift_px[1] = 0.f;
            res->sw2sq = __int_as_float(0x7fc00000);
            res->status = status;
        }
        if (curve)
            for (int l = t; l < NN; l += 256) curve[l] = __int_as_float(0x7fc00000);
        return;
    }
    const float *U = a.ref_qt + r * (int64_t)Q * NN;
    const float *V = a.img_qt + gi * (int64_t)Q * NN;
    for (int i = t; i < NN; i += 256) Dbits[i] = 0u;
    float uacc = 0.f, vacc = 0.f;  // thread t < NN: column energies of U and V
    f32x4m acc[RA][NB];
#pragma unroll
    for (int ra = 0; ra < RA; ++ra)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[ra][b] = f32x4m{0.f, 0.f, 0.f, 0.f};
    const bool rows_live = wave < NB;  // NN = 64: every wave owns one row block
    for (int j0 = 0; j0 < Q; j0 += KC) {
        __syncthreads();
        for (int q = t; q < KC * (NN / 4); q += 256) {
            const int jr = q / (NN / 4), c4 = q - jr * (NN / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j0 + jr < Q) v = *(const float4 *)(V + (int64_t)(j0 + jr) * NN + 4 * c4);
            *(float4 *)(vs + jr * VS + 4 * c4) = v;
        }
        __syncthreads();
        if (t < NN) {
            for (int jr = 0; jr < KC && j0 + jr < Q; ++jr) {
                const float x = vs[jr * VS + t];
                const float u = U[(int64_t)(j0 + jr) * NN + t];
                vacc = fmaf(x, x, vacc);
                uacc = fmaf(u, u, uacc);
            }
        }
        if (rows_live) {
            // A fragments: A[i][kk] = U[j0 + 4 s + kk][16 a + i]
            float afr[RA][KC / 4];
#pragma unroll
            for (int ra = 0; ra < RA; ++ra) {
                const int ab = wave + 4 * ra;
#pragma unroll
                for (int s = 0; s < KC / 4; ++s) {
                    const int j = j0 + 4 * s + lk;
                    afr[ra][s] = j < Q && ab < NB ? U[(int64_t)j * NN + 16 * ab + li] : 0.f;
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int s = 0; s < KC / 4; ++s) {
                    // B[kk][jj] = V[j0 + 4 s + kk][16 b + jj]
                    const float bfr = vs[(4 * s + lk) * VS + 16 * b + li];
#pragma unroll
                    for (int ra = 0; ra < RA; ++ra)
                        acc[ra][b] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(afr[ra][s], bfr, acc[ra][b], 0, 0, 0);
                }
            }
        }
    }
    if (t < NN) {
        uu[t] = uacc;
        vv[t] = vacc;
    }
    __syncthreads();
    // residual of column k at lag (k' - k) mod n, max over k by atomics
    const float invQ = 1.f / (float)Q;
    if (rows_live) {
#pragma unroll
        for (int ra = 0; ra < RA; ++ra) {
            const int ab = wave + 4 * ra;
            if (ab >= NB) continue;  // wave-uniform
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * ab + 4 * lk + e, kp = 16 * b + li;
                    const float v = fmaxf((uu[k] + vv[kp] - 2.f * acc[ra][b][e]) * invQ, 0.f);
                    const int lag = kp >= k ? kp - k : kp - k + NN;
                    atomicMax(&Dbits[lag], __float_as_uint(v));
                }
            }
        }
    }
    __syncthreads();
    if (curve)
        for (int l = t; l < NN; l += 256) curve[l] = __uint_as_float(Dbits[l]);
    // top_k lags of the estimate (wave 0; ties to the smaller lag)
    const int K = a.top_k;
    if (wave == 0) {
        float v0 = lane < NN ? __uint_as_float(Dbits[lane]) : __builtin_inff();
        float v1 = lane + 64 < NN ? __uint_as_float(Dbits[lane + 64]) : __builtin_inff();
        for (int c = 0; c < K; ++c) {
            float v = v0;
            int i = lane;
            if (v1 < v) {
                v = v1;
                i = lane + 64;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const float v2 = __shfl_xor(v, off, 64);
                const int i2 = __shfl_xor(i, off, 64);
                if (v2 < v || (v2 == v && i2 < i)) {
                    v = v2;
                    i = i2;
                }
            }
            if (lane == 0) cand[c] = i;
            if (i == lane) v0 = __builtin_inff();
            if (i == lane + 64) v1 = __builtin_inff();
        }
    }
    __syncthreads();
    // rescore: direct FP32 column residuals at every candidate, max over k
    // (threads past TPC n idle)
    constexpr int TPC = 256 / NN;  // threads per column
    const int k = t % NN, part = t / NN;
    for (int c = 0; c < K; ++c) {
        const int l = cand[c];
        const float *Vc = V + (k + l < NN ? k + l : k + l - NN);
        float s = 0.f;
        if (part < TPC)
            for (int j = part; j < Q; j += TPC) {
                const float d = U[(int64_t)j * NN + k] - Vc[(int64_t)j * NN];
                s = fmaf(d, d, s);
            }
        colred[t] = s;
        __syncthreads();
        if (t < NN) {
            float col = 0.f;
            for (int p2 = 0; p2 < TPC; ++p2) col += colred[p2 * NN + t];
            colred[t] = col;
        }
        __syncthreads();
        if (wave == 0) {
            float m = fmaxf(lane < NN ? colred[lane] : 0.f, lane + 64 < NN ? colred[lane + 64] : 0.f);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
            if (lane == 0) cval[c] = m * invQ;
        }
        __syncthreads();
    }
    if (t == 0) {
        int bl = cand[0];
        float bv = cval[0];
        for (int c = 1; c < K; ++c)
            if (cval[c] < bv || (cval[c] == bv && cand[c] < bl)) {
                bv = cval[c];
                bl = cand[c];
            }
        res->rot_index = bl;
        res->theta_rad = (float)(6.283185307179586 * (double)bl / (double)NN);
        res->shift_px[0] = res->shift_px[1] = 0.f;
        res->sw2sq = bv;
        res->status = 0;
    }
}

bool msw_supported(Geo g) { return g.n % 16 == 0 && g.n <= 128; }

template <int NN>
static void launch_msw_t(const PairArgs &a, Geo g, int64_t P, hipStream_t s) {
    hipLaunchKernelGGL((k_align_msw<NN>), dim3((unsigned)P), dim3(256), 0, s, a, g);
}

hipError_t launch_align_msw(const PairArgs &a, Geo g, hipStream_t s) {
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (P <= 0) return hipSuccess;
    switch (g.n) {  // the admissible n (factors 2 and 3) that are multiples of 16 up to 128
    case 16: launch_msw_t<16>(a, g, P, s); break;
    case 32: launch_msw_t<32>(a, g, P, s); break;
    case 48: launch_msw_t<48>(a, g, P, s); break;
    case 64: launch_msw_t<64>(a, g, P, s); break;
    case 96: launch_msw_t<96>(a, g, P, s); break;
    case 128: launch_msw_t<128>(a, g, P, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sw
