// CDFs and quantile tables (Sec. 2.3: cumulative sums of each projection,
// then the inverse CDF by linear interpolation; generalised inverse
// inf{t : F(t) >= z} of App. A).
//
// One block per image, one wave per column at a time.  A column of L <= 256
// bins is held as up to four values per lane; the mass and the cumulative
// sums are accumulated in FP64 (lane-local sums, then a wave-wide DPP scan of
// the lane totals), so each lane holds the normalised CDF at the right edges
// of its own bins.  Levels are then assigned from the bins' side rather than
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
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
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

// Number of levels z_j <= c, for z_j = (j + 1/2)/Q (midpoint) or j/Q
// (left): floor(c Q + 1/2) or floor(c Q) + 1, clamped to [0, Q].  Monotone
// in c, so the counts at consecutive bin edges partition the levels; a level
// that ties an edge to within rounding lands on either side of it, where the
// interpolated quantile is the same edge value.
__device__ __forceinline__ int levels_at_or_below(double c, int Q, double zshift) {
    const int j = (int)fma(c, (double)Q, zshift);  // truncation = floor for c >= 0
    return min(max(j, 0), Q);
}

// h / den for den > 0: hardware reciprocal and two Newton steps (FP64).
__device__ __forceinline__ double div_by(double h, double den) {
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    return h * r;
}

// Invert one column, M bins per lane (M = ceil(L / 64)).  `col` reads bin b
// of the column (FP32).  Writes the quantile of every level j into
// Ut[j * ldt + kl] and returns the lane's partial (sum of quantiles, sum of
// squares) in *su, *sq, and the column mass (same value on all lanes).
template <int M, typename ColFn>
__device__ double invert_column_m(ColFn col, int L, int Q, int levels, float *Ut, int ldt, int kl,
                                  int lane, double *su, double *sq) {
    double v[M];
    double run = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const int b = lane * M + t;
        double x = 0.0;
        if (b < L) x = (double)col(b);
        run += x;
        v[t] = run;  // lane-local inclusive sums
    }
    const double excl = wave_inclusive_scan_d(run) - run;
    // mass = cumulative sum at the last bin, taken from the lane holding it
    const int last_lane = (L - 1) / M;
    const int last_t = (L - 1) - last_lane * M;
    double lastv = v[0];
#pragma unroll
    for (int t = 1; t < M; ++t)
        if (t == last_t) lastv = v[t];
    const double mass = read_lane_d(excl + lastv, last_lane);
    const double h = 2.0 / (double)L;
    const double invQ = 1.0 / (double)Q;
    const double z0 = levels ? 0.0 : 0.5 * invQ;       // z_j = j / Q + z0
    const double zshift = levels ? 1.0 : 0.5;           // level count offset
    double s1 = 0.0, s2 = 0.0;
    if (!(mass > 0.0)) {
        // empty (or non-finite) column: the inverse of a zero CDF, as in the
        // lower-bound rule with every CDF value 0
        for (int j = lane; j < Q; j += 64) {
            const int b = (levels && j == 0) ? 0 : L - 1;
            const float uf = (float)(-1.0 + (double)b * h);
            Ut[j * ldt + kl] = uf;
            s1 += (double)uf;
            s2 += (double)uf * (double)uf;
        }
    } else {
        const double invm = 1.0 / mass;
        double c[M];
#pragma unroll
        for (int t = 0; t < M; ++t) c[t] = (excl + v[t]) * invm;  // C at the right edge of bin
        // the CDF reaches exactly 1 at the right edge of the last bin
#pragma unroll
        for (int t = 0; t < M; ++t)
            if (lane * M + t == L - 1) c[t] = 1.0;
        // C at the left edge of this lane's first bin: the previous lane's
        // last right edge (0 on lane 0)
        const double cm = c[M - 1];
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(cm), 0x138, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(cm), 0x138, 0xf, 0xf, false);
        double cl = __hiloint2double(hi, lo);  // wave_shr:1
        int jl = lane == 0 ? 0 : levels_at_or_below(cl, Q, zshift);
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int b = lane * M + t;
            if (b < L) {
                const double cr = c[t];
                const int jr = levels_at_or_below(cr, Q, zshift);
                const double tl = fma((double)b, h, -1.0), tr = tl + h;
                const double den = cr - cl;
                const double slope = den > 0.0 ? div_by(h, den) : 0.0;
                // the offset z - cl inside the bin in FP64, the interpolation
                // and the clamp to the bin in FP32 (the result's precision)
                const float tlf = (float)tl, trf = (float)tr, slf = (float)slope;
                for (int j = jl; j < jr; ++j) {
                    const double z = fma((double)j, invQ, z0);
                    const float uf =
                        __builtin_amdgcn_fmed3f(fmaf((float)(z - cl), slf, tlf), tlf, trf);
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

template <typename ColFn>
__device__ __forceinline__ double invert_column(ColFn col, int L, int Q, int levels, float *Ut,
                                                int ldt, int kl, int lane, double *su,
                                                double *sq) {
    const int m = (L + 63) >> 6;  // bins per lane, <= 4 (wave-uniform)
    if (m == 1) return invert_column_m<1>(col, L, Q, levels, Ut, ldt, kl, lane, su, sq);
    if (m == 2) return invert_column_m<2>(col, L, Q, levels, Ut, ldt, kl, lane, su, sq);
    if (m == 3) return invert_column_m<3>(col, L, Q, levels, Ut, ldt, kl, lane, su, sq);
    return invert_column_m<4>(col, L, Q, levels, Ut, ldt, kl, lane, su, sq);
}

// The whole CDF/quantile phase of one image, shared by the stand-alone,
// fused and mixed kernels.  col(k, b) reads bin b of column k.  LDS: Ut
// (Q * (TC + 1) floats), colS (2 n doubles).
// Column sums are stored per column and reduced by wave 0 in a fixed order,
// so the per-image scalars do not depend on the block size or tile width.
template <int NT, typename ColFn>
__device__ void quantile_phase(ColFn col, int L, int n, int Q, int levels, int TC,
                               const double2 *__restrict__ d64, float *Ut, double *colS,
                               float *__restrict__ U, double *__restrict__ A) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ldt = TC + 1;
    double mass0 = 0.0;
    for (int k0 = 0; k0 < n; k0 += TC) {
        for (int kl = wave; kl < TC; kl += NW) {
            const int k = k0 + kl;
            double su, sq;
            const double mass = invert_column([&](int b) { return col(k, b); }, L, Q, levels, Ut,
                                              ldt, kl, lane, &su, &sq);
            if (k == 0) mass0 = mass;
            su = wave_sum_d(su);
            sq = wave_sum_d(sq);
            if (lane == 0) {
                colS[2 * k] = su;
                colS[2 * k + 1] = sq;
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < Q * TC; idx += NT) {
            const int j = idx / TC, kl = idx - j * TC;
            U[(int64_t)j * n + k0 + kl] = Ut[j * ldt + kl];
        }
        __syncthreads();
    }
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
