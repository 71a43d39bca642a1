// CDFs and quantile tables (Sec. 2.3: cumulative sums of each projection,
// then the inverse CDF by linear interpolation; generalised inverse
// inf{t : F(t) >= z} of App. A).
//
// One block per image, one wave per column at a time.  A column of L <= 256
// bins is held as up to four values per lane; the mass and the cumulative
// sums are accumulated in FP64 (lane-local sums, then a wave-wide exclusive
// scan of the lane totals) and the normalised CDF is kept in a per-wave LDS
// buffer.  Each lane then inverts the CDF at its quantile levels by binary
// search (lower bound: first bin whose CDF reaches z) and linear
// interpolation inside that bin.  Quantiles are gathered in an LDS tile
// [Q][TC] and written out as rows of the [Q][n] table (angle fastest).  The
// per-image scalars (mass, E = sum of squares, translation moment a) are
// reduced in FP64 on the way.
#pragma once
#include "sw_internal.h"

namespace sw {

template <int NT>
struct QuantShape {
    int L, n, Q, levels, TC;
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Inclusive scan over the 64 lanes of a wave (Hillis-Steele).
__device__ __forceinline__ double wave_inclusive_scan_d(double v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Invert one column.  `col` reads bin b of the column (FP32).  Writes the
// quantiles of levels j = lane, lane + 64, ... into Ut[j * ldt + kl] and
// returns the lane's partial (sum of quantiles, sum of squares) in *su, *sq.
// Returns the column mass (same value on all lanes).
template <typename ColFn>
__device__ double invert_column(ColFn col, int L, int Q, int levels, double *C, float *Ut, int ldt,
                                int kl, int lane, double *su, double *sq) {
    const int m = (L + 63) >> 6;  // bins per lane, <= 4
    double v[4];
    double run = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = lane * m + t;
        double x = 0.0;
        if (t < m && b < L) x = (double)col(b);
        run += x;
        v[t] = run;  // lane-local inclusive sums
    }
    const double incl = wave_inclusive_scan_d(run, lane);
    const double excl = incl - run;
    // mass = cumulative sum at the last bin, taken from the lane holding it,
    // so that C[L-1] is exactly 1
    const int last_lane = (L - 1) / m;
    const int last_t = (L - 1) - last_lane * m;
    double lastv = v[0];
#pragma unroll
    for (int t = 1; t < 4; ++t)
        if (t == last_t) lastv = v[t];
    const double mass = __shfl(excl + lastv, last_lane, 64);
    const bool pos = mass > 0.0;
    if (lane == 0) C[0] = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = lane * m + t;
        if (t < m && b < L) C[b + 1] = pos ? (excl + v[t]) / mass : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double h = 2.0 / (double)L;
    double s1 = 0.0, s2 = 0.0;
    for (int j = lane; j < Q; j += 64) {
        const double z = levels ? (double)j / (double)Q : ((double)j + 0.5) / (double)Q;
        int lo = 0, hi = L;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (C[mid + 1] >= z) hi = mid;
            else lo = mid + 1;
        }
        const int b = lo < L ? lo : L - 1;
        const double tl = -1.0 + (double)b * h, tr = -1.0 + (double)(b + 1) * h;
        const double den = C[b + 1] - C[b];
        double u = den > 0.0 ? tl + h * (z - C[b]) / den : tl;
        u = u < tl ? tl : (u > tr ? tr : u);
        const float uf = (float)u;
        Ut[j * ldt + kl] = uf;
        s1 += (double)uf;
        s2 += (double)uf * (double)uf;
    }
    *su = s1;
    *sq = s2;
    __builtin_amdgcn_wave_barrier();
    return mass;
}

inline int pick_tc(int n, int Q, size_t budget) {
    const int cands[4] = {64, 32, 16, 8};
    for (int c : cands)
        if (n % c == 0 && (size_t)Q * (c + 1) * 4 <= budget) return c;
    return 8;
}

}  // namespace sw
