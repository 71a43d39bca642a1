// CDFs and quantile tables (Sec. 2.3: cumulative sums of each projection,
// then the inverse CDF by linear interpolation; generalised inverse
// inf{t : F(t) >= z} of App. A).
//
// One block per image.  A column is inverted by half a wave (32 lanes, two
// columns per wave at a time) for L <= 128 and by a whole wave for larger L,
// so a lane holds at most four bins.  The mass and the cumulative sums are
// accumulated in FP64 (lane-local sums, then a DPP scan of the lane totals
// across the half or the wave), so each lane holds the normalised CDF at the
// right edges of its own bins.  Levels are then assigned from the bins' side rather than
// searched for: level z_j falls in the first bin whose right-edge CDF reaches
// it, so a lane counts the levels at or below each of its edges and
// interpolates the levels in between.  Quantiles
// are gathered in an LDS tile [Q][TC] and written out as rows of the [Q][n]
// table (angle fastest).  The per-image scalars (mass, E = sum of squares,
// translation moment a) are reduced in FP64 on the way.
#pragma once
#include "sw_internal.h"

namespace sw {

template <int NT>
struct QuantShape {
    int L, n, Q, levels, TC;
};

// v moved across lanes by a DPP control (row_mask selects the 16-lane rows
// that receive; lanes without a valid source, and rows not selected, get 0).
// With every row selected the bound control supplies the zeros, so no
// zeroed destination has to be set up first.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
    if (ROWS == 0xf) {
        const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
        const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
        return __hiloint2double(hi, lo);
    }
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Inclusive scan over the 64 lanes of a wave: shifts by 1, 2, 4, 8 inside
// each row of 16 lanes, then the row totals carried across rows.  Fixed
// summation order, so the result is deterministic.
__device__ __forceinline__ double wave_inclusive_scan_d(double v) {
    v += dpp_d<0x111, 0xf>(v);  // row_shr:1
    v += dpp_d<0x112, 0xf>(v);  // row_shr:2
    v += dpp_d<0x114, 0xf>(v);  // row_shr:4
    v += dpp_d<0x118, 0xf>(v);  // row_shr:8
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ double read_lane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the wave (same value on all lanes).
__device__ __forceinline__ double wave_sum_d(double v) {
    return read_lane_d(wave_inclusive_scan_d(v), 63);
}

// Inclusive scan within each half (lanes 0-31, 32-63) of the wave: shifts
// by 1, 2, 4, 8 inside each row of 16 lanes, then the first row's total of
// each half carried into its second row.  Fixed order, deterministic.
__device__ __forceinline__ double half_inclusive_scan_d(double v) {
    v += dpp_d<0x111, 0xf>(v);  // row_shr:1
    v += dpp_d<0x112, 0xf>(v);  // row_shr:2
    v += dpp_d<0x114, 0xf>(v);  // row_shr:4
    v += dpp_d<0x118, 0xf>(v);  // row_shr:8
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    return v;
}

// Lane hl of this lane's group (the half `half` of the wave, or the wave).
template <bool HALF>
__device__ __forceinline__ double read_group_lane_d(double v, int hl, int half) {
    if (!HALF) return read_lane_d(v, hl);
    const double a = read_lane_d(v, hl), b = read_lane_d(v, 32 + hl);
    return half ? b : a;
}

template <bool HALF>
__device__ __forceinline__ double group_inclusive_scan_d(double v) {
    return HALF ? half_inclusive_scan_d(v) : wave_inclusive_scan_d(v);
}

// Sum over this lane's group (same value on the group's lanes).
template <bool HALF>
__device__ __forceinline__ double group_sum_d(double v, int half) {
    return read_group_lane_d<HALF>(group_inclusive_scan_d<HALF>(v), HALF ? 31 : 63, half);
}

// Number of levels z_j <= c, for z_j = (j + 1/2)/Q (midpoint) or j/Q
// (left): floor(c Q + 1/2) or floor(c Q) + 1, clamped to [0, Q].  Monotone
// in c, so the counts at consecutive bin edges partition the levels; a level
// that ties an edge to within rounding lands on either side of it, where the
// interpolated quantile is the same edge value.
__device__ __forceinline__ int levels_at_or_below(double c, int Q, double zshift) {
    const int j = (int)fma(c, (double)Q, zshift);  // truncation = floor for c >= 0
    return min(max(j, 0), Q);
}

// 1 / m for m > 0: hardware reciprocal and two Newton steps (FP64).
__device__ __forceinline__ double recip_d(double m) {
    double r = __builtin_amdgcn_rcp(m);
    r = fma(r, fma(-m, r, 1.0), r);
    r = fma(r, fma(-m, r, 1.0), r);
    return r;
}

// h / den in FP32 for den > 0 (the interpolation runs in FP32): the FP64 CDF
// step rounded to FP32, its hardware reciprocal refined by one Newton step.
__device__ __forceinline__ float slope_f(float h, double den) {
    const float d = (float)den;
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaf(r, fmaf(-d, r, 1.f), r);
    return h * r;
}

// Invert one column with a group of G lanes (G = 32: the half `half` of the
// wave; G = 64: the whole wave), M = ceil(L / G) bins per lane; lane hl of
// the group holds bins hl M .. hl M + M - 1.  `col` reads bin b of the column
// (FP32).  Writes the quantile of every level j into Ut[j * ldt + kl] and
// returns the lane's partial (sum of quantiles, sum of squares) in *su, *sq,
// and the column mass (same value on the group's lanes).
template <int M, bool HALF, typename ColFn>
__device__ double invert_column_m(ColFn col, int L, int Q, int levels, float *Ut, int ldt, int kl,
                                  int hl, int half, double *su, double *sq) {
    constexpr int G = HALF ? 32 : 64;
    // the lane's M bins read at once (bins past the column read the last
    // bin and are dropped), then summed
    float xs[M];
#pragma unroll
    for (int t = 0; t < M; ++t) xs[t] = col(min(hl * M + t, L - 1));
    double v[M];
    double run = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        run += hl * M + t < L ? (double)xs[t] : 0.0;
        v[t] = run;  // lane-local inclusive sums
    }
    const double excl = group_inclusive_scan_d<HALF>(run) - run;
    // mass = cumulative sum at the last bin, taken from the lane holding it
    const int last_lane = (L - 1) / M;
    const int last_t = (L - 1) - last_lane * M;
    double lastv = v[0];
#pragma unroll
    for (int t = 1; t < M; ++t)
        if (t == last_t) lastv = v[t];
    const double mass = read_group_lane_d<HALF>(excl + lastv, last_lane, half);
    const double h = 2.0 / (double)L;
    const double invQ = 1.0 / (double)Q;
    const double z0 = levels ? 0.0 : 0.5 * invQ;       // z_j = j / Q + z0
    const double zshift = levels ? 1.0 : 0.5;           // level count offset
    double s1 = 0.0, s2 = 0.0;
    if (!(mass > 0.0)) {
        // empty (or non-finite) column: the inverse of a zero CDF, as in the
        // lower-bound rule with every CDF value 0
        for (int j = hl; j < Q; j += G) {
            const int b = (levels && j == 0) ? 0 : L - 1;
            const float uf = (float)(-1.0 + (double)b * h);
            Ut[j * ldt + kl] = uf;
            s1 += (double)uf;
            s2 += (double)uf * (double)uf;
        }
    } else {
        const double invm = recip_d(mass);
        // C at the right edge of bin b = hl M + t; exactly 1 at the last bin
        auto cdf = [&](int t) {
            return hl * M + t == L - 1 ? 1.0 : (excl + v[t]) * invm;
        };
        // C at the left edge of this lane's first bin: the previous lane's
        // last right edge (0 on the first lane of the group)
        double cl = dpp_d<0x138, 0xf>(cdf(M - 1));  // wave_shr:1
        if (hl == 0) cl = 0.0;  // with halves, lane 32 got lane 31's edge
        int jl = hl == 0 ? 0 : levels_at_or_below(cl, Q, zshift);
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int b = hl * M + t;
            if (b < L) {
                const double cr = cdf(t);
                const int jr = levels_at_or_below(cr, Q, zshift);
                const double tl = fma((double)b, h, -1.0), tr = tl + h;
                const double den = cr - cl;
                // the offset z - cl inside the bin in FP64 (advanced by 1/Q
                // per level), the slope, the interpolation and the clamp to
                // the bin in FP32 (the result's precision)
                const float tlf = (float)tl, trf = (float)tr;
                const float slf = den > 0.0 ? slope_f((float)h, den) : 0.f;
                double zc = fma((double)jl, invQ, z0) - cl;
                for (int j = jl; j < jr; ++j, zc += invQ) {
                    const float uf = __builtin_amdgcn_fmed3f(fmaf((float)zc, slf, tlf), tlf, trf);
                    Ut[j * ldt + kl] = uf;
                    s1 += (double)uf;
                    s2 = fma((double)uf, (double)uf, s2);
                }
                cl = cr;
                jl = jr;
            }
        }
    }
    *su = s1;
    *sq = s2;
    __builtin_amdgcn_wave_barrier();
    return mass;
}

// HALF: L <= 128; otherwise 128 < L <= 256.  Either way M <= 4.
template <bool HALF, typename ColFn>
__device__ __forceinline__ double invert_column(ColFn col, int L, int Q, int levels, float *Ut,
                                                int ldt, int kl, int hl, int half, double *su,
                                                double *sq) {
    const int m = HALF ? (L + 31) >> 5 : (L + 63) >> 6;  // bins per lane (wave-uniform)
    switch (m) {
    case 1: return invert_column_m<1, HALF>(col, L, Q, levels, Ut, ldt, kl, hl, half, su, sq);
    case 2: return invert_column_m<2, HALF>(col, L, Q, levels, Ut, ldt, kl, hl, half, su, sq);
    case 3: return invert_column_m<3, HALF>(col, L, Q, levels, Ut, ldt, kl, hl, half, su, sq);
    default: return invert_column_m<4, HALF>(col, L, Q, levels, Ut, ldt, kl, hl, half, su, sq);
    }
}

// Invert the TC columns k0 .. k0 + TC - 1 of a tile: with halves, columns
// 2 p and 2 p + 1 go to the two halves of wave p (TC is even).
template <int NT, bool HALF, typename ColFn>
__device__ __forceinline__ void invert_tile(ColFn col, int L, int Q, int levels, int TC, int k0,
                                            float *Ut, double *colS, double *mass0) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hl = HALF ? lane & 31 : lane, half = HALF ? lane >> 5 : 0;
    const int per_wave = HALF ? 2 : 1;
    for (int p = wave; per_wave * p < TC; p += NW) {
        const int kl = per_wave * p + half, k = k0 + kl;
        double su, sq;
        const double mass = invert_column<HALF>([&](int b) { return col(k, b); }, L, Q, levels,
                                                Ut, TC + 1, kl, hl, half, &su, &sq);
        if (k == 0) *mass0 = mass;
        su = group_sum_d<HALF>(su, half);
        sq = group_sum_d<HALF>(sq, half);
        if (hl == 0) {
            colS[2 * k] = su;
            colS[2 * k + 1] = sq;
        }
    }
}

// All tiles of columns of one image: invert a tile into Ut, then write it
// out as rows of the [Q][n] table (angle fastest).  Returns the mass of
// column 0 (on the lanes that inverted it).
template <int NT, bool HALF, typename ColFn>
__device__ double quantile_tiles(ColFn col, int L, int n, int Q, int levels, int TC, float *Ut,
                                 double *colS, float *__restrict__ U) {
    const int ldt = TC + 1;
    double mass0 = 0.0;
    for (int k0 = 0; k0 < n; k0 += TC) {
        invert_tile<NT, HALF>(col, L, Q, levels, TC, k0, Ut, colS, &mass0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < Q * TC; idx += NT) {
            const int j = idx / TC, kl = idx - j * TC;
            U[(int64_t)j * n + k0 + kl] = Ut[j * ldt + kl];
        }
        __syncthreads();
    }
    return mass0;
}

// Which column inversion a kernel compiles: both, chosen by L at run time,
// or only the half-wave one (the caller guarantees L <= 128) or only the
// whole-wave one (L > 128).  A kernel that keeps other values live across
// the phase compiles one, so that its registers are those of one body.
enum QuantMode { kQuantAuto = 0, kQuantHalf = 1, kQuantWave = 2 };

__host__ __device__ inline QuantMode quant_mode_for(int L) {
    return L <= 128 ? kQuantHalf : kQuantWave;
}

// The whole CDF/quantile phase of one image, shared by the stand-alone,
// fused and mixed kernels.  col(k, b) reads bin b of column k.  LDS: Ut
// (Q * (TC + 1) floats), colS (2 n doubles).
// Column sums are stored per column and reduced by wave 0 in a fixed order,
// so the per-image scalars do not depend on the block size or tile width.
template <int NT, int QM = kQuantAuto, typename ColFn>
__device__ void quantile_phase(ColFn col, int L, int n, int Q, int levels, int TC,
                               const double2 *__restrict__ d64, float *Ut, double *colS,
                               float *__restrict__ U, double *__restrict__ A) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double mass0;
    if (QM == kQuantHalf || (QM == kQuantAuto && L <= 128))
        mass0 = quantile_tiles<NT, true>(col, L, n, Q, levels, TC, Ut, colS, U);
    else
        mass0 = quantile_tiles<NT, false>(col, L, n, Q, levels, TC, Ut, colS, U);
    if (wave == 0) {
        double e = 0.0, x = 0.0, y = 0.0;
        for (int k = lane; k < n; k += 64) {
            const double qbar = colS[2 * k] / (double)Q;
            const double2 d = d64[k];
            e += colS[2 * k + 1];
            x += qbar * d.x;
            y += qbar * d.y;
        }
        e = wave_sum_d(e);
        x = wave_sum_d(x);
        y = wave_sum_d(y);
        if (lane == 0 && A) {
            A[0] = mass0;  // column 0 is inverted by wave 0
            A[1] = e;
            A[2] = x / (double)n;
            A[3] = y / (double)n;
        }
    }
    __syncthreads();
}

inline int pick_tc(int n, int Q, size_t budget) {
    const int cands[4] = {64, 32, 16, 8};
    for (int c : cands)
        if (n % c == 0 && (size_t)Q * (c + 1) * 4 <= budget) return c;
    return 8;
}

}  // namespace sw
