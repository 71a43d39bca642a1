// Kernels and launchers of the n = 128 alignment; the device routines are in
// align128_dev.h.
#include "align128_dev.h"

namespace sw {

// Coefficients of every reference: gam[r][p][slot] and gamx[r][p][0..1]
// (see gamma128_coef).  spec: FP32 spectra [n_ref][65][Q].
__global__ __launch_bounds__(256) void k_gamma128(const float2 *__restrict__ spec, int64_t n_ref,
                                                  int Q, float2 *__restrict__ gam,
                                                  float2 *__restrict__ gamx) {
    const int P2 = Q / 2;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n_ref * P2 * (kA128Slots + 2)) return;
    const int slot = (int)(idx % (kA128Slots + 2));
    const int64_t rp = idx / (kA128Slots + 2);
    const int p = (int)(rp % P2);
    const int64_t r = rp / P2;
    const float2 c = gamma128_coef(spec + r * 65 * (int64_t)Q, Q, p, slot);
    if (slot < kA128Slots) gam[rp * kA128Slots + slot] = c;
    else gamx[rp * 2 + (slot - kA128Slots)] = c;
}

// BF16: the launch's a.bf16, one instance each so that either has its own
// register allocation.
template <int NT, bool BF16>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_align128(
    PairArgs a, Geo g, const float2 *__restrict__ gam, const float2 *__restrict__ gamx,
    const float2 *__restrict__ tw32, const double2 *__restrict__ tw64) {
    __shared__ A128Lds<NT> sm;
    const int Q = g.Q, P2 = Q / 2;
    const int64_t pi = blockIdx.x;
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (pi >= P) return;
    const int64_t r = a.pairs ? a.pairs[2 * pi] : pi / a.n_img;
    const int64_t gi = a.pairs ? a.pairs[2 * pi + 1] : pi % a.n_img;
    const bool in_range = r >= 0 && r < a.n_ref && gi >= 0 && gi < a.n_img;
    const int64_t rr = in_range ? r : 0, gg = in_range ? gi : 0;
    A128Job job;
    job.U = a.ref_qt + rr * (int64_t)Q * 128;
    job.V = a.img_qt + gg * (int64_t)Q * 128;
    job.au = a.ref_aux + 4 * rr;
    job.av = a.img_aux + 4 * gg;
    job.G = gam + rr * (int64_t)P2 * kA128Slots;
    job.GX = gamx + rr * (int64_t)P2 * 2;
    job.d32 = tw32;
    job.d64 = tw64;
    job.res = a.out + pi;
    job.curve = a.curve ? a.curve + pi * 128 : nullptr;
    job.Q = Q;
    job.L = g.L;
    job.mode = a.mode;
    job.bf16 = a.bf16;
    job.top_k = a.top_k;
    int status = 0;
    if (!in_range) status = 3;  // bad pair index
    else if (isnan(job.au[0]) || isnan(job.av[0])) status = 2;
    else if (!(job.au[0] > 0.0) || !(job.av[0] > 0.0)) status = 1;
    job.status = status;
    align128_pair<NT, BF16>(job, sm);
}

// One pair per wave (align128_wave): NW waves per block share the angle table.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_align128w(
    PairArgs a, Geo g, const float2 *__restrict__ gam, const float2 *__restrict__ gamx,
    const float2 *__restrict__ tw32, const double2 *__restrict__ tw64) {
    __shared__ float2 tw[128];
    __shared__ __attribute__((aligned(16))) float2 wl[NW * kA128WaveElems];
    for (int i = threadIdx.x; i < 128; i += 64 * NW) tw[i] = tw32[i];
    __syncthreads();
    // the wave index made uniform, so that the pair's pointers live in
    // scalar registers
    const int Q = g.Q, P2 = Q / 2, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t pi = (int64_t)blockIdx.x * NW + wave;
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (pi >= P) return;  // wave-uniform; no block barrier follows
    const int64_t r = a.pairs ? a.pairs[2 * pi] : pi / a.n_img;
    const int64_t gi = a.pairs ? a.pairs[2 * pi + 1] : pi % a.n_img;
    const bool in_range = r >= 0 && r < a.n_ref && gi >= 0 && gi < a.n_img;
    const int64_t rr = in_range ? r : 0, gg = in_range ? gi : 0;
    A128Job job;
    job.U = a.ref_qt + rr * (int64_t)Q * 128;
    job.V = a.img_qt + gg * (int64_t)Q * 128;
    job.au = a.ref_aux + 4 * rr;
    job.av = a.img_aux + 4 * gg;
    job.G = gam + rr * (int64_t)P2 * kA128Slots;
    job.GX = gamx + rr * (int64_t)P2 * 2;
    job.d32 = tw32;
    job.d64 = tw64;
    job.res = a.out + pi;
    job.curve = a.curve ? a.curve + pi * 128 : nullptr;
    job.Q = Q;
    job.L = g.L;
    job.mode = a.mode;
    job.bf16 = a.bf16;
    job.top_k = a.top_k;
    int status = 0;
    if (!in_range) status = 3;  // bad pair index
    else if (isnan(job.au[0]) || isnan(job.av[0])) status = 2;
    else if (!(job.au[0] > 0.0) || !(job.av[0] > 0.0)) status = 1;
    job.status = status;
    align128_wave(job, wl + wave * kA128WaveElems, tw);
}

bool align128_supported(Geo g) { return g.n == 128; }

size_t align128_scratch_bytes(Geo g, int64_t n_ref) {
    const size_t per = sizeof(float2) * (size_t)(g.Q / 2) * (kA128Slots + 2);
    return per * (size_t)n_ref;
}

hipError_t launch_align128(const PairArgs &a, Geo g, const AngleTable &t, float2 *gam,
                           hipStream_t s, bool per_wave) {
    const int64_t P = a.pairs ? a.n_pairs : a.n_ref * a.n_img;
    if (P <= 0) return hipSuccess;
    float2 *gamx = gam + (size_t)a.n_ref * (g.Q / 2) * kA128Slots;
    const int64_t ng = a.n_ref * (g.Q / 2) * (kA128Slots + 2);
    hipLaunchKernelGGL(k_gamma128, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, a.ref_spec,
                       a.n_ref, g.Q, gam, gamx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (per_wave) {
        constexpr int NW = 4;  // 38 KiB of LDS: four blocks per compute unit
        hipLaunchKernelGGL((k_align128w<NW>), dim3((unsigned)((P + NW - 1) / NW)), dim3(64 * NW), 0,
                           s, a, g, gam, gamx, t.d32, t.d64);
        return hipGetLastError();
    }
    constexpr int NT = 256;  // 4 waves, four blocks per compute unit
    if (a.bf16)
        hipLaunchKernelGGL((k_align128<NT, true>), dim3((unsigned)P), dim3(NT), 0, s, a, g, gam,
                           gamx, t.d32, t.d64);
    else
        hipLaunchKernelGGL((k_align128<NT, false>), dim3((unsigned)P), dim3(NT), 0, s, a, g, gam,
                           gamx, t.d32, t.d64);
    return hipGetLastError();
}

}  // namespace sw
