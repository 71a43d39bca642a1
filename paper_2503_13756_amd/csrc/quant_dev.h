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

// The whole CDF/quantile phase of one image, shared by the stand-alone,
// fused and mixed kernels.  col(k, b) reads bin b of column k.  LDS: C
// (NW * (L + 1) doubles), Ut (Q * (TC + 1) floats), colS (2 n doubles).
// Column sums are stored per column and reduced by wave 0 in a fixed order,
// so the per-image scalars do not depend on the block size or tile width.
template <int NT, typename ColFn>
__device__ void quantile_phase(ColFn col, int L, int n, int Q, int levels, int TC,
                               const double2 *__restrict__ d64, double *C0, float *Ut,
                               double *colS, float *__restrict__ U, double *__restrict__ A) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *C = C0 + wave * (L + 1);
    const int ldt = TC + 1;
    double mass0 = 0.0;
    for (int k0 = 0; k0 < n; k0 += TC) {
        for (int kl = wave; kl < TC; kl += NW) {
            const int k = k0 + kl;
            double su, sq;
            const double mass = invert_column([&](int b) { return col(k, b); }, L, Q, levels, C,
                                              Ut, ldt, kl, lane, &su, &sq);
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
