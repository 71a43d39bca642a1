// Complex multiply and batched Stockham FFTs in LDS with radix 4, 3 and 2
// (lengths 2^a 3^b), shared by the per-pair alignment (angle FFTs) and the
// Fourier-slice projector (lengths that are not powers of two).
#pragma once
#include "sw_internal.h"

namespace sw {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int R>
__device__ __forceinline__ void dft_small(float2 (&a)[R]) {
    if constexpr (R == 2) {
        const float2 x = a[0], y = a[1];
        a[0] = make_float2(x.x + y.x, x.y + y.y);
        a[1] = make_float2(x.x - y.x, x.y - y.y);
    } else if constexpr (R == 4) {
        const float2 t0 = make_float2(a[0].x + a[2].x, a[0].y + a[2].y);
        const float2 t1 = make_float2(a[0].x - a[2].x, a[0].y - a[2].y);
        const float2 t2 = make_float2(a[1].x + a[3].x, a[1].y + a[3].y);
        const float2 t3 = make_float2(a[1].x - a[3].x, a[1].y - a[3].y);
        a[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        a[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        a[1] = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - i t3
        a[3] = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + i t3
    } else {  // R == 3, w = e^{-2 pi i / 3}
        const float h3 = 0.86602540378443864676f;
        const float2 s = make_float2(a[1].x + a[2].x, a[1].y + a[2].y);
        const float2 d = make_float2(a[1].x - a[2].x, a[1].y - a[2].y);
        const float2 m = make_float2(a[0].x - 0.5f * s.x, a[0].y - 0.5f * s.y);
        a[0] = make_float2(a[0].x + s.x, a[0].y + s.y);
        a[1] = make_float2(m.x + h3 * d.y, m.y - h3 * d.x);
        a[2] = make_float2(m.x - h3 * d.y, m.y + h3 * d.x);
    }
}

// One Stockham pass of radix R over `rows` complex rows of length n, from X
// to Y (row stride n).  p = product of the radices already applied.
template <int NT, int R>
__device__ void fft_pass(const float2 *X, float2 *Y, int rows, int n, int p, const float2 *tw) {
    const int nr = n / R;
    const int nb = rows * nr;
    const int ts = n / (p * R);
    for (int idx = threadIdx.x; idx < nb; idx += NT) {
        const int row = idx / nr, i = idx - row * nr;
        const int k = i % p;
        const float2 *x = X + row * n + i;
        float2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            v[q] = x[q * nr];
            if (q > 0) v[q] = cmul(v[q], tw[q * k * ts]);
        }
        dft_small<R>(v);
        float2 *y = Y + row * n + (i - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) y[q * p] = v[q];
    }
    __syncthreads();
}

// Forward FFT of `rows` rows held in A; B is a buffer of the same size.
// Returns the buffer holding the result.
template <int NT>
__device__ float2 *fft_rows(float2 *A, float2 *B, int rows, int n, const float2 *tw) {
    int p = 1, m = n;
    float2 *x = A, *y = B;
    while (m % 4 == 0) {
        fft_pass<NT, 4>(x, y, rows, n, p, tw);
        p *= 4; m /= 4;
        float2 *t = x; x = y; y = t;
    }
    while (m % 3 == 0) {
        fft_pass<NT, 3>(x, y, rows, n, p, tw);
        p *= 3; m /= 3;
        float2 *t = x; x = y; y = t;
    }
    while (m % 2 == 0) {
        fft_pass<NT, 2>(x, y, rows, n, p, tw);
        p *= 2; m /= 2;
        float2 *t = x; x = y; y = t;
    }
    return x;
}

}  // namespace sw
