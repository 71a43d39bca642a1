// Host runtime of libswalign: contexts, geometry checks, angle tables,
// scratch, and the C entry points declared in include/swalign.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <regex>
#include <sstream>
#include <string>
#include <vector>

#include "host_internal.h"

namespace swh {

thread_local std::string g_err;

const std::string &last_error() { return g_err; }

sw_status fail(sw_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

sw_status hip_fail(hipError_t e, const char *where) {
    return fail(SW_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}



bool only_2_3(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

sw_status check_geom(const sw_geom *g, sw::Geo *out) {
    if (!g) return fail(SW_E_INVALID, "geometry pointer is NULL");
    if (g->L < 8 || g->L > sw::kMaxL)
        return fail(SW_E_INVALID, "L = %d outside [8, %d]", g->L, sw::kMaxL);
    if (g->n_angles < 8 || g->n_angles > sw::kMaxN || g->n_angles % 8 != 0 || !only_2_3(g->n_angles))
        return fail(SW_E_INVALID,
                    "n_angles = %d must be a multiple of 8 in [8, %d] with prime factors 2 and 3 only",
                    g->n_angles, sw::kMaxN);
    if (g->n_quantiles < 8 || g->n_quantiles > sw::kMaxQ || g->n_quantiles % 4 != 0)
        return fail(SW_E_INVALID, "n_quantiles = %d must be a multiple of 4 in [8, %d]",
                    g->n_quantiles, sw::kMaxQ);
    if (g->levels != SW_LEVELS_MIDPOINT && g->levels != SW_LEVELS_LEFT)
        return fail(SW_E_INVALID, "levels = %d is not a sw_levels value", g->levels);
    out->L = g->L;
    out->n = g->n_angles;
    out->Q = g->n_quantiles;
    out->levels = g->levels;
    return SW_OK;
}

// (cos theta_m, -sin theta_m) for theta_m = 2 pi m / n.  The first octant is
// evaluated in FP64; the rest follows from reflection about pi/4 and quarter
// turns, so the symmetries the projection kernel relies on hold exactly.
void angle_values(int n, std::vector<double> &c, std::vector<double> &s) {
    c.assign(n, 0.0);
    s.assign(n, 0.0);
    const int q = n / 4, o = n / 8;
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m <= o; ++m) {
        c[m] = std::cos(two_pi * m / n);
        s[m] = std::sin(two_pi * m / n);
    }
    c[0] = 1.0;
    s[0] = 0.0;
    for (int m = o + 1; m < q; ++m) {  // theta_m = pi/2 - theta_{q-m}
        c[m] = s[q - m];
        s[m] = c[q - m];
    }
    for (int m = q; m < n; ++m) {  // theta_m = theta_{m-q} + pi/2
        c[m] = -s[m - q];
        s[m] = c[m - q];
    }
}

sw_status get_table(Ctx *ctx, int n, const sw::AngleTable **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tables.find(n);
    if (it != ctx->tables.end()) {
        *out = &it->second;
        return SW_OK;
    }
    std::vector<double> c, s;
    angle_values(n, c, s);
    std::vector<float2> t32(n);
    std::vector<double2> t64(n);
    for (int m = 0; m < n; ++m) {
        t32[m] = make_float2((float)c[m], (float)(-s[m]));
        t64[m] = make_double2(c[m], -s[m]);
    }
    sw::AngleTable t;
    t.n = n;
    hipError_t e = hipMalloc(&t.d32, sizeof(float2) * n);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(angle table)");
    e = hipMalloc(&t.d64, sizeof(double2) * n);
    if (e != hipSuccess) {
        (void)hipFree(t.d32);
        return hip_fail(e, "hipMalloc(angle table)");
    }
    e = hipMemcpy(t.d32, t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.d64, t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t.d32);
        (void)hipFree(t.d64);
        return hip_fail(e, "hipMemcpy(angle table)");
    }
    auto res = ctx->tables.emplace(n, t);
    *out = &res.first->second;
    return SW_OK;
}

// ---- the allocation-free alignment entry point (sw_align_batch_noalloc) ----
// Its device memory is one file-scope array per GPU: the angle tables of every
// admissible n_angles (written once per device at set-up) followed by the
// work area that sw_align_batch takes from the context scratch (reference
// spectra and n = 128 coefficients, or the bfloat16 spectra and candidate
// lags of the all-pairs path).  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress, per device.
constexpr size_t kNoAllocAngleBytes = 128 * 1024;
constexpr size_t kNoAllocWorkBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocAngleBytes + kNoAllocWorkBytes];

struct NoAllocDevice {
    sw_status status = SW_OK;  // of the set-up on this device
    std::string err;
    char *work = nullptr;      // device address of the work area
    std::map<int, sw::AngleTable> tables;
};
static std::mutex g_noalloc_mu;
static std::map<int, NoAllocDevice> g_noalloc;  // per device

// Set-up on the current device (once per device): the array's device
// address, and the angle tables of every admissible n copied into it.
static void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc.count(device)) return;
    NoAllocDevice &d = g_noalloc[device];
    char *base = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&base, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !base) {
        d.status = SW_E_DEVICE;
        d.err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    size_t off = 0;
    for (int n = 8; n <= sw::kMaxN; n += 8) {
        if (!only_2_3(n)) continue;
        std::vector<double> c, sn;
        angle_values(n, c, sn);
        std::vector<float2> t32(n);
        std::vector<double2> t64(n);
        for (int m = 0; m < n; ++m) {
            t32[m] = make_float2((float)c[m], (float)(-sn[m]));
            t64[m] = make_double2(c[m], -sn[m]);
        }
        sw::AngleTable t;
        t.n = n;
        t.d64 = (double2 *)(base + off);
        off += sizeof(double2) * n;
        t.d32 = (float2 *)(base + off);
        off += (sizeof(float2) * n + 15) & ~(size_t)15;
        if (off > kNoAllocAngleBytes) {
            d.status = SW_E_DEVICE;
            d.err = "angle tables exceed their part of the no-alloc scratch";
            return;
        }
        e = hipMemcpy(t.d64, t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(t.d32, t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            d.status = SW_E_DEVICE;
            d.err = std::string("hipMemcpy(no-alloc angle tables): ") + hipGetErrorString(e);
            return;
        }
        d.tables[n] = t;
    }
    d.work = base + kNoAllocAngleBytes;
}

static sw_status noalloc_device(int device, NoAllocDevice **out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc.find(device);
    if (it == g_noalloc.end())
        return fail(SW_E_INVALID, "the no-alloc scratch of device %d is not set up", device);
    if (it->second.status != SW_OK) return fail(it->second.status, "%s", it->second.err.c_str());
    *out = &it->second;
    return SW_OK;
}

// Work order of the projection for (L, n): every (slot, bin) item gets the
// range of image rows where a pixel inside the disk has non-zero weight for
// its line (pixel (i, j) weighs 1 - c |j - u(i)| with u(i) the column where
// the line crosses row i; a small margin keeps the range conservative under
// FP32 rounding).  Units of 8 consecutive bins of one slot take the union of
// their items' ranges, units are ordered by the centre of their range, and
// each run of eight forms a task; a local search then swaps units between
// tasks while that does not lengthen the two tasks' ranges together (fixed
// seed: the plan is a function of (L, n)).  Rows outside a task's range only
// ever add zeros, so skipping them leaves every sum unchanged, whatever the
// plan.
static void build_plan(int L, int n, std::vector<int> &perm, std::vector<int2> &trow) {
    std::vector<double> c, s;
    angle_values(n, c, s);
    const int slots = n / 8 + 1, upr = (L + 7) / 8, ntasks = sw::proj_ntasks(L, n);
    const double c0 = 0.5 * (L - 1);
    const int r = L - 2;
    struct Unit {
        int slot, b0, lo, hi;
    };
    std::vector<Unit> units;
    for (int k = 0; k < slots; ++k) {
        const double ck = c[k], sk = s[k], half = 1.0 / ck + 1e-3;
        for (int u0 = 0; u0 < upr; ++u0) {
            int lo = L, hi = -1;
            for (int b = 8 * u0; b < std::min(L, 8 * u0 + 8); ++b) {
                for (int i = 0; i < L; ++i) {
                    if (i >= lo && i <= hi) continue;  // already in the unit's range
                    const double u = (b - c0 + sk * (i - c0)) / ck + c0;
                    const int ja = std::max(0, (int)std::floor(u - half));
                    const int jb = std::min(L - 1, (int)std::ceil(u + half));
                    const int bb = 2 * i - L + 1;
                    for (int j = ja; j <= jb; ++j) {
                        const int a = 2 * j - L + 1;
                        if (a * a + bb * bb <= r * r && ck * std::fabs(j - u) < 1.0 + 1e-3) {
                            lo = std::min(lo, i);
                            hi = std::max(hi, i);
                            break;
                        }
                    }
                }
            }
            units.push_back(Unit{k, 8 * u0, lo, hi});
        }
    }
    // units whose lines miss the disk first, then by the centre of the range
    std::stable_sort(units.begin(), units.end(), [](const Unit &x, const Unit &y) {
        const int kx = x.lo <= x.hi ? x.lo + x.hi : -1, ky = y.lo <= y.hi ? y.lo + y.hi : -1;
        return kx < ky;
    });
    // local search: task t holds units[8 t .. 8 t + 7]; a swap is kept when
    // the two tasks' range lengths do not grow in sum
    const int nu = (int)units.size();
    auto span = [&](int t) {
        int lo = L, hi = -1;
        for (int q = 8 * t; q < std::min(nu, 8 * t + 8); ++q)
            if (units[q].lo <= units[q].hi) {
                lo = std::min(lo, units[q].lo);
                hi = std::max(hi, units[q].hi);
            }
        return hi >= lo ? hi - lo + 1 : 0;
    };
    if (ntasks > 1) {
        std::vector<int> len(ntasks);
        for (int t = 0; t < ntasks; ++t) len[t] = span(t);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        auto next = [&](int m) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            return (int)((st >> 33) % (uint64_t)m);
        };
        const long iters = 200000 + 50L * nu;
        for (long it = 0; it < iters; ++it) {
            const int qa = next(nu), qb = next(nu);
            const int ta = qa / 8, tb = qb / 8;
            if (ta == tb) continue;
            std::swap(units[qa], units[qb]);
            const int la = span(ta), lb = span(tb);
            if (la + lb <= len[ta] + len[tb]) {
                len[ta] = la;
                len[tb] = lb;
            } else {
                std::swap(units[qa], units[qb]);
            }
        }
    }
    perm.assign((size_t)ntasks * 64, -1);
    trow.assign(ntasks, make_int2(1, 0));
    for (size_t q = 0; q < units.size(); ++q) {
        const Unit &x = units[q];
        const int t = (int)(q / 8), l0 = (int)(q % 8) * 8;
        for (int l = 0; l < 8 && x.b0 + l < L; ++l) perm[(size_t)t * 64 + l0 + l] = x.slot * L + x.b0 + l;
        if (x.lo <= x.hi) {
            int2 &tr = trow[t];
            if (tr.x > tr.y) tr = make_int2(x.lo, x.hi);
            else tr = make_int2(std::min(tr.x, x.lo), std::max(tr.y, x.hi));
        }
    }
}

sw_status get_plan(Ctx *ctx, int L, int n, const sw::ProjPlan **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int key = L * 4096 + n;
    auto f = ctx->plans.find(key);
    if (f != ctx->plans.end()) {
        *out = &f->second;
        return SW_OK;
    }
    std::vector<int> perm;
    std::vector<int2> trow;
    build_plan(L, n, perm, trow);
    sw::ProjPlan p;
    p.L = L;
    p.n = n;
    p.ntasks = (int)trow.size();
    hipError_t e = hipMalloc(&p.perm, sizeof(int) * perm.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(projection plan)");
    e = hipMalloc(&p.trow, sizeof(int2) * trow.size());
    if (e != hipSuccess) {
        (void)hipFree(p.perm);
        return hip_fail(e, "hipMalloc(projection plan)");
    }
    e = hipMemcpy(p.perm, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.trow, trow.data(), sizeof(int2) * trow.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p.perm);
        (void)hipFree(p.trow);
        return hip_fail(e, "hipMemcpy(projection plan)");
    }
    auto res = ctx->plans.emplace(key, p);
    *out = &res.first->second;
    return SW_OK;
}

// Cyclic kernel of the ramp filter |w| sampled on M = 2L frequencies (DC
// zero): h[0] = M/4, h[m] = -1/(M sin^2(pi m / M)) for odd m, 0 for even
// m != 0.  Stored as hx[t] = h[t - (LP - 1)] for |t - (LP - 1)| < L, zero
// elsewhere, t < 2 LP - 1 (the layout launch_ramp reads).
static sw_status get_ramp_table(Ctx *ctx, int L, const float **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto f = ctx->ramp_tables.find(L);
    if (f != ctx->ramp_tables.end()) {
        *out = f->second;
        return SW_OK;
    }
    const int LP = sw::ramp_padded_length(L), M = 2 * L;
    std::vector<float> hx(2 * LP - 1, 0.f);
    const double pi = 3.141592653589793238462643383279502884;
    for (int t = 0; t < 2 * LP - 1; ++t) {
        const int m = t - (LP - 1);
        if (m <= -L || m >= L) continue;
        const int mm = ((m % M) + M) % M;
        double v = 0.0;
        if (mm == 0) v = M / 4.0;
        else if (mm & 1) {
            const double sn = std::sin(pi * mm / M);
            v = -1.0 / (M * sn * sn);
        }
        hx[t] = (float)v;
    }
    float *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(float) * hx.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(ramp table)");
    e = hipMemcpy(d, hx.data(), sizeof(float) * hx.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "hipMemcpy(ramp table)");
    }
    ctx->ramp_tables.emplace(L, d);
    *out = d;
    return SW_OK;
}

// Tables of the Fourier-slice projector for L (even, factors 2 and 3), laid out as
// described beside sw::FourierTabs in one device buffer.  The interpolation
// kernel is the exponential of semicircle phi(z) = exp(beta (sqrt(1 -
// (2z/W)^2) - 1)), |z| < W/2, on the grid oversampled by 2; its Fourier
// transform phihat(zeta) = int phi(z) cos(2 pi zeta z) dz is integrated in
// FP64 after z = (W/2) sin t, which leaves a smooth periodic integrand for
// the midpoint rule.
static constexpr float kFourierBeta = 2.3f * (float)sw::kFourierW;

static double es_hat(double zeta) {
    const double pi = 3.141592653589793238462643383279502884;
    const int nodes = 512;
    const double W = (double)sw::kFourierW, beta = (double)kFourierBeta;
    double acc = 0.0;
    for (int q = 0; q < nodes; ++q) {
        const double t = -0.5 * pi + (q + 0.5) * pi / nodes;
        acc += std::exp(beta * (std::cos(t) - 1.0)) * std::cos(t) *
               std::cos(pi * zeta * W * std::sin(t));
    }
    return 0.5 * W * (pi / nodes) * acc;
}

static sw_status get_fourier_tabs(Ctx *ctx, int L, sw::FourierTabs *out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int M = L / 2, Nf = 2 * L;
    const size_t n2 = (size_t)Nf + L + L;  // float2 entries
    auto f = ctx->fourier_tabs.find(L);
    void *d = nullptr;
    if (f != ctx->fourier_tabs.end()) {
        d = f->second;
    } else {
        const double pi = 3.141592653589793238462643383279502884;
        std::vector<float2> t2(n2);
        std::vector<float> corr(L);
        for (int k = 0; k < Nf; ++k)
            t2[k] = make_float2((float)std::cos(2 * pi * k / Nf), (float)-std::sin(2 * pi * k / Nf));
        for (int k = 0; k < L; ++k)
            t2[Nf + k] = make_float2((float)std::cos(2 * pi * k / L), (float)-std::sin(2 * pi * k / L));
        for (int t = 0; t < L; ++t) {
            const int k = t < M ? t : t - L;
            const double sg = (k & 1) ? -1.0 : 1.0;
            t2[Nf + L + t] =
                make_float2((float)(sg * std::cos(pi * k / L)), (float)(sg * std::sin(pi * k / L)));
        }
        for (int j = 0; j < L; ++j) corr[j] = (float)(1.0 / es_hat((double)(j - M) / Nf));
        hipError_t e = hipMalloc(&d, sizeof(float2) * n2 + sizeof(float) * L);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(Fourier tables)");
        e = hipMemcpy(d, t2.data(), sizeof(float2) * n2, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char *)d + sizeof(float2) * n2, corr.data(), sizeof(float) * L,
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(e, "hipMemcpy(Fourier tables)");
        }
        ctx->fourier_tabs.emplace(L, d);
    }
    const float2 *t2 = (const float2 *)d;
    out->twf = t2;
    out->twl = t2 + Nf;
    out->shift = t2 + Nf + L;
    out->corr = (const float *)(t2 + n2);
    return SW_OK;
}

static double es_phi(double z) {
    const double W = (double)sw::kFourierW, t = 2.0 * z / W;
    return std::fabs(t) < 1.0 ? std::exp((double)kFourierBeta * (std::sqrt(1.0 - t * t) - 1.0))
                              : 0.0;
}

// Slice-point table of the Fourier-slice projector for L and the slice
// directions d = (c[m], -s[m]): for each slice m and k = 0 .. L/2, the
// fine-grid point g = k d Nf / L of the slice frequency k pi d (mirrored to
// g_x >= 0, the conjugate then taken in the kernel), its first tap row u0
// and column v0 of the kernel's support, the kernel weights per row and
// column, and the factor exp(-i pi k (d_x + d_y) / L) sinc(pi k d_x / L)
// sinc(pi k d_y / L) (the pixel centres' half-pixel offset and the transform
// of one pixel cell), all from FP64.  Layout as read by slice_point in
// k_fourier.hip.
static std::vector<float4> fourier_target_table(int L, const std::vector<double> &c,
                                                const std::vector<double> &s) {
    const double pi = 3.141592653589793238462643383279502884;
    const int M = L / 2, Nf = 2 * L, W = sw::kFourierW, nsl = (int)c.size();
    std::vector<float4> tab((size_t)nsl * (M + 1) * 5);
    for (int m = 0; m < nsl; ++m) {
        const double dx = c[m], dy = -s[m];
        const bool flip = dx < 0.0;
        for (int k = 0; k <= M; ++k) {
            const double sc = (double)k * Nf / L;
            const double gx = (flip ? -dx : dx) * sc, gy = (flip ? -dy : dy) * sc;
            const int v0 = (int)std::floor(gx - 0.5 * W) + 1, u0 = (int)std::floor(gy - 0.5 * W) + 1;
            float wx[8] = {0}, wy[8] = {0};
            for (int t = 0; t < W; ++t) {
                wx[t] = (float)es_phi(gx - (v0 + t));
                wy[t] = (float)es_phi(gy - (u0 + t));
            }
            const double ax = pi * k * dx / L, ay = pi * k * dy / L, ang = -(ax + ay);
            const double sinc = (ax == 0.0 ? 1.0 : std::sin(ax) / ax) * (ay == 0.0 ? 1.0 : std::sin(ay) / ay);
            float4 *e = &tab[((size_t)m * (M + 1) + k) * 5];
            int hdr[2] = {((u0 % Nf) + Nf) % Nf, (v0 + sw::kFourierPad) | (flip ? 1 << 16 : 0)};
            float hf[2];
            std::memcpy(hf, hdr, sizeof(hf));
            e[0] = make_float4(hf[0], hf[1], (float)(std::cos(ang) * sinc), (float)(std::sin(ang) * sinc));
            e[1] = make_float4(wx[0], wx[1], wx[2], wx[3]);
            e[2] = make_float4(wx[4], wx[5], wx[6], 0.f);
            e[3] = make_float4(wy[0], wy[1], wy[2], wy[3]);
            e[4] = make_float4(wy[4], wy[5], wy[6], 0.f);
        }
    }
    return tab;
}

static sw_status upload_table(const std::vector<float4> &tab, void **d) {
    hipError_t e = hipMalloc(d, sizeof(float4) * tab.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(Fourier slice table)");
    e = hipMemcpy(*d, tab.data(), sizeof(float4) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(*d);
        return hip_fail(e, "hipMemcpy(Fourier slice table)");
    }
    return SW_OK;
}

// Table for the grid angles theta_m = 2 pi m / n, m < n/2 (the kernel writes
// the theta + pi mirrors).
static sw_status get_fourier_targets(Ctx *ctx, int L, int n, const float4 **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int key = L * 4096 + n;
    auto f = ctx->fourier_targets.find(key);
    if (f != ctx->fourier_targets.end()) {
        *out = (const float4 *)f->second;
        return SW_OK;
    }
    std::vector<double> c, s;
    angle_values(n, c, s);
    c.resize(n / 2);
    s.resize(n / 2);
    void *d = nullptr;
    sw_status st = upload_table(fourier_target_table(L, c, s), &d);
    if (st != SW_OK) return st;
    ctx->fourier_targets.emplace(key, d);
    *out = (const float4 *)d;
    return SW_OK;
}

// Slice-point table and direction table (cos theta, -sin theta) for n
// explicit angles (radians), cached by the angles' exact bytes.
static sw_status get_fourier_dir_targets(Ctx *ctx, int L, int n, const double *theta,
                                         const float4 **out, const sw::AngleTable **dirs) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::string key((const char *)&L, sizeof(int));
    key.append((const char *)theta, sizeof(double) * n);
    auto f = ctx->fourier_dir_targets.find(key);
    if (f != ctx->fourier_dir_targets.end()) {
        *out = (const float4 *)f->second;
        *dirs = &ctx->fourier_dir_angles.at(key);
        return SW_OK;
    }
    std::vector<double> c(n), s(n);
    std::vector<float2> t32(n);
    std::vector<double2> t64(n);
    for (int m = 0; m < n; ++m) {
        c[m] = std::cos(theta[m]);
        s[m] = std::sin(theta[m]);
        t32[m] = make_float2((float)c[m], (float)(-s[m]));
        t64[m] = make_double2(c[m], -s[m]);
    }
    void *d = nullptr;
    sw_status st = upload_table(fourier_target_table(L, c, s), &d);
    if (st != SW_OK) return st;
    sw::AngleTable t;
    t.n = n;
    hipError_t e = hipMalloc(&t.d32, sizeof(float2) * n);
    if (e == hipSuccess) {
        e = hipMalloc(&t.d64, sizeof(double2) * n);
        if (e != hipSuccess) (void)hipFree(t.d32);
    }
    if (e == hipSuccess) {
        e = hipMemcpy(t.d32, t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(t.d64, t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(t.d32);
            (void)hipFree(t.d64);
        }
    }
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "direction table");
    }
    ctx->fourier_dir_targets.emplace(key, d);
    auto it = ctx->fourier_dir_angles.emplace(key, t).first;
    *out = (const float4 *)d;
    *dirs = &it->second;
    return SW_OK;
}

static int log2_exact(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return (1 << l) == v ? l : -1;
}

sw_status get_scratch(Ctx *ctx, size_t bytes, hipStream_t stream, void **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (bytes > ctx->scratch_bytes) {
        if (ctx->scratch) {
            // the old buffer may still be in use by work queued on the stream
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(ctx->scratch);
            ctx->scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        size_t sz = bytes + bytes / 4;
        hipError_t e = hipMalloc(&ctx->scratch, sz);
        if (e != hipSuccess) return fail(SW_E_NOMEM, "hipMalloc(%zu) for scratch failed", sz);
        ctx->scratch_bytes = sz;
    }
    *out = ctx->scratch;
    return SW_OK;
}

// Pinned descriptor slot for one mixed launch (two groups: refs, images).
sw_status ring_slot(Ctx *c, sw::MixGroup **host) {
    DescRing &r = c->ring;
    const int i = r.next;
    r.next = (r.next + 1) % DescRing::kSlots;
    if (r.used[i]) {
        hipError_t e = hipEventSynchronize(r.ev[i]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(descriptor slot)");
    }
    r.used[i] = true;
    *host = r.host + 2 * i;
    return SW_OK;
}
hipEvent_t ring_event(Ctx *c, sw::MixGroup *host) {
    return c->ring.ev[(host - c->ring.host) / 2];
}

// Align up to kMaxMix stacks in one set of mixed launches.  Stacks must be
// validated.  R_override > 0 forces the projection strip rows, and knobs (if
// given) the launch knobs (autotuner); otherwise the context's tuned values.
sw_status run_stack_chunk(Ctx *c, const sw_stack *const *st, int n, int mode, int bf16, int top_k,
                          int R_override, hipStream_t s, const sw::MixKnobs *knobs = nullptr) {
    sw::MixGroup *hg;
    sw_status stt = ring_slot(c, &hg);
    if (stt != SW_OK) return stt;
    sw::MixGroup &gr = hg[0], &gi = hg[1];
    gr.nitems = gi.nitems = n;
    gr.total = gi.total = 0;
    // items aligned by the n = 128 register-FFT kernel first (work items
    // [0, split)), the rest after
    auto fast_geom = [&](const sw_stack &k) {
        return k.geom.n_angles == 128 && !c->generic_align;
    };
    std::vector<int> order;
    for (int i = 0; i < n; ++i)
        if (fast_geom(*st[i])) order.push_back(i);
    const int nfast = (int)order.size();
    for (int i = 0; i < n; ++i)
        if (!fast_geom(*st[i])) order.push_back(i);
    int64_t first = 0, split = 0;
    for (int ii = 0; ii < n; ++ii) {
        const int i = ii;
        const sw_stack &k = *st[order[ii]];
        sw::Geo geo{k.geom.L, k.geom.n_angles, k.geom.n_quantiles, k.geom.levels};
        const sw::AngleTable *t;
        if ((stt = get_table(c, geo.n, &t)) != SW_OK) return stt;
        const sw::ProjPlan *pp;
        if ((stt = get_plan(c, geo.L, geo.n, &pp)) != SW_OK) return stt;
        sw::MixItem a{};
        a.perm = pp->perm;
        a.trow = pp->trow;
        a.L = geo.L;
        a.n = geo.n;
        a.Q = geo.Q;
        a.levels = geo.levels;
        auto tr = c->tile_R.find(geo.L);
        a.R = R_override > 0 ? R_override : (tr != c->tile_R.end() ? tr->second : 0);
        a.d32 = t->d32;
        a.d64 = t->d64;
        a.mode = mode;
        a.bf16 = bf16;
        a.top_k = top_k;
        a.ref_qt = k.ref_qt;
        a.ref_aux = k.ref_aux;
        sw::MixItem r = a;
        r.img = k.ref_img;
        r.qt = k.ref_qt;
        r.aux = k.ref_aux;
        r.first = i;
        r.count = 1;
        a.img = k.imgs;
        a.qt = k.qt;
        a.aux = k.aux;
        a.out = (sw::Result *)k.out;
        a.first = first;
        a.count = k.N;
        a.gam = nullptr;
        r.gam = nullptr;
        a.spec = r.spec = 1;  // the reference item writes the spectrum
        first += k.N;
        if (i < nfast) split = first;
        gr.items[i] = r;
        gi.items[i] = a;
    }
    gr.total = n;
    gi.total = first;
    gr.split = 0;
    gi.split = split;
    std::vector<std::pair<int, int64_t>> sizes;
    for (int i = 0; i < n; ++i) sizes.emplace_back(gi.items[i].L, gi.items[i].count);
    sw::MixLaunch m = sw::plan_mixed(gi.items, n, knobs ? *knobs : c->knobs_for(sizes));
    for (int i = 0; i < n; ++i) {
        gr.items[i].R = gi.items[i].R;
        gr.items[i].TC = gi.items[i].TC;
        gr.items[i].fused = gi.items[i].fused;
    }
    // device scratch: two groups, counters, reference spectra, PMF slots
    const int grid = 2 * c->cu_count;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_groups = take(2 * sizeof(sw::MixGroup));
    const size_t o_cnt = take(4 * sizeof(unsigned long long));
    std::vector<size_t> o_spec(n), o_gam(n);
    for (int i = 0; i < n; ++i) {
        const sw::Geo gg{gi.items[i].L, gi.items[i].n, gi.items[i].Q, gi.items[i].levels};
        o_spec[i] = take(sizeof(float2) * (size_t)(gi.items[i].n / 2 + 1) * gi.items[i].Q);
        o_gam[i] = i < nfast ? take(sw::align128_scratch_bytes(gg, 1)) : 0;
    }
    const size_t o_slots = take(sizeof(float) * (size_t)m.slot_floats * grid);
    void *scr;
    if ((stt = get_scratch(c, off, s, &scr)) != SW_OK) return stt;
    char *base = (char *)scr;
    for (int i = 0; i < n; ++i) {
        gi.items[i].ref_spec = (float2 *)(base + o_spec[i]);
        gr.items[i].ref_spec = gi.items[i].ref_spec;
        if (i < nfast) gi.items[i].gam = (float2 *)(base + o_gam[i]);
    }
    sw::MixGroup *d_groups = (sw::MixGroup *)(base + o_groups);
    hipError_t e = hipMemcpyAsync(d_groups, hg, 2 * sizeof(sw::MixGroup), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ring_event(c, hg), s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    e = sw::launch_mixed(d_groups, d_groups + 1, m, (unsigned long long *)(base + o_cnt),
                         (float *)(base + o_slots), grid, s);
    return e == hipSuccess ? SW_OK : hip_fail(e, "mixed launch");
}

Ctx *as_ctx(void *p) { return static_cast<Ctx *>(p); }

}  // namespace swh

using namespace swh;

extern "C" {

const char *sw_last_error(void) { return g_err.c_str(); }

const char *sw_version(void) { return "swalign 0.1 (gfx950)"; }

sw_status sw_projection_plan(int32_t L, int32_t n, int32_t cap_tasks, int32_t *perm,
                             int32_t *row_lo, int32_t *row_hi, int32_t *ntasks) {
    if (!ntasks) return fail(SW_E_INVALID, "ntasks out-pointer is NULL");
    if (L < 8 || L > sw::kMaxL) return fail(SW_E_INVALID, "L = %d outside [8, %d]", L, sw::kMaxL);
    if (n < 8 || n > sw::kMaxN || n % 8 != 0)
        return fail(SW_E_INVALID, "n = %d is not a multiple of 8 in [8, %d]", n, sw::kMaxN);
    const int nt = sw::proj_ntasks(L, n);
    *ntasks = nt;
    if (cap_tasks == 0 && !perm && !row_lo && !row_hi) return SW_OK;
    if (cap_tasks < nt || !perm || !row_lo || !row_hi)
        return fail(SW_E_INVALID, "the plan of (L = %d, n = %d) has %d tasks (cap %d)", L, n, nt,
                    cap_tasks);
    std::vector<int> pv;
    std::vector<int2> tr;
    build_plan(L, n, pv, tr);
    for (size_t i = 0; i < pv.size(); ++i) perm[i] = pv[i];
    for (int t = 0; t < nt; ++t) {
        row_lo[t] = tr[t].x;
        row_hi[t] = tr[t].y;
    }
    return SW_OK;
}

sw_status sw_ctx_create(void **ctx, int device, const char *tune_json) {
    (void)tune_json;
    if (!ctx) return fail(SW_E_INVALID, "ctx out-pointer is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(SW_E_INVALID, "device %d not in [0, %d)", device, count);
    Ctx *c = new (std::nothrow) Ctx;
    if (!c) return fail(SW_E_NOMEM, "out of host memory");
    c->device = device;
    {
        DeviceGuard dg(device);
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            cu > 0)
            c->cu_count = cu;
        e = hipHostMalloc((void **)&c->ring.host, sizeof(sw::MixGroup) * 2 * DescRing::kSlots);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipHostMalloc(descriptor ring)");
        }
        for (int i = 0; i < DescRing::kSlots; ++i)
            if ((e = hipEventCreateWithFlags(&c->ring.ev[i], hipEventDisableTiming)) != hipSuccess) {
                delete c;
                return hip_fail(e, "hipEventCreate");
            }
        // the no-alloc entry point's scratch on this device (a failure is
        // reported by that entry point, every other call works without it)
        noalloc_setup(device);
    }
    if (tune_json && *tune_json) {
        std::ifstream f(tune_json);
        if (!f) {
            delete c;
            return fail(SW_E_INVALID, "cannot read tile table %s", tune_json);
        }
        std::stringstream ss;
        ss << f.rdbuf();
        const std::string txt = ss.str();
        // "L": {"R": rows[, "tpw": tasks][, "align_bpc": blocks] ...}
        const std::regex re("\"(\\d+)\"\\s*:\\s*\\{\\s*\"R\"\\s*:\\s*(\\d+)"
                            "(\\s*,\\s*\"tpw\"\\s*:\\s*(\\d+))?"
                            "(\\s*,\\s*\"align_bpc\"\\s*:\\s*(\\d+))?");
        for (auto it = std::sregex_iterator(txt.begin(), txt.end(), re); it != std::sregex_iterator();
             ++it) {
            const int L = std::stoi((*it)[1]);
            c->tile_R[L] = std::stoi((*it)[2]);
            if ((*it)[4].matched) c->tile_tpw[L] = std::stoi((*it)[4]);
            if ((*it)[6].matched) c->tile_abpc[L] = std::stoi((*it)[6]);
        }
        std::smatch m;
        if (std::regex_search(txt, m, std::regex("\"small_batch\"\\s*:\\s*(\\d+)")))
            c->small_batch = std::stoi(m[1]);
        if (std::regex_search(txt, m, std::regex("\"align_kernel\"\\s*:\\s*\"generic\"")))
            c->generic_align = true;
        if (std::regex_search(txt, m, std::regex("\"align_kernel\"\\s*:\\s*\"block128\"")))
            c->align128_per_wave = false;
        if (std::regex_search(txt, m, std::regex("\"tables_images_per_block\"\\s*:\\s*([12])")))
            c->tables_per_block = std::stoi(m[1]);
        if (std::regex_search(txt, m, std::regex("\"serve_fail_ticket\"\\s*:\\s*(\\d+)")))
            c->serve_fail_ticket = std::stoull(m[1]);
    }
    *ctx = c;
    return SW_OK;
}

sw_status sw_ctx_destroy(void *ctx) {
    if (!ctx) return SW_OK;
    Ctx *c = as_ctx(ctx);
    stop_server(c);
    {
        DeviceGuard dg(c->device);
        (void)hipDeviceSynchronize();
        for (auto &kv : c->tables) {
            (void)hipFree(kv.second.d32);
            (void)hipFree(kv.second.d64);
        }
        for (auto &kv : c->plans) {
            (void)hipFree(kv.second.perm);
            (void)hipFree(kv.second.trow);
        }
        for (auto &kv : c->ramp_tables) (void)hipFree(kv.second);
        for (auto &kv : c->fourier_tabs) (void)hipFree(kv.second);
        for (auto &kv : c->fourier_targets) (void)hipFree(kv.second);
        for (auto &kv : c->fourier_dir_targets) (void)hipFree(kv.second);
        for (auto &kv : c->fourier_dir_angles) {
            (void)hipFree(kv.second.d32);
            (void)hipFree(kv.second.d64);
        }
        if (c->scratch) (void)hipFree(c->scratch);
        for (int i = 0; i < DescRing::kSlots; ++i)
            if (c->ring.ev[i]) (void)hipEventDestroy(c->ring.ev[i]);
        if (c->ring.host) (void)hipHostFree(c->ring.host);
    }
    delete c;
    return SW_OK;
}

sw_status sw_project(void *ctx, const float *img, int64_t N, const sw_geom *g, float *pmf,
                     void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!img || !pmf) return fail(SW_E_INVALID, "img or pmf is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    const sw::ProjPlan *pp;
    if ((st = get_plan(c, geo.L, geo.n, &pp)) != SW_OK) return st;
    hipError_t e = sw::launch_project(img, N, geo, *t, *pp, pmf, (hipStream_t)stream,
                                      c->small(N));
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_project launch");
}

sw_status sw_quantiles(void *ctx, const float *pmf, int64_t N, const sw_geom *g, float *qt,
                       double *aux, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!pmf || !qt) return fail(SW_E_INVALID, "pmf or qt is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    hipError_t e = sw::launch_quantiles(pmf, N, geo, *t, qt, aux, (hipStream_t)stream,
                                        c->small(N));
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_quantile launch");
}

sw_status sw_tables(void *ctx, const float *img, int64_t N, const sw_geom *g, float *qt,
                    double *aux, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!img || !qt) return fail(SW_E_INVALID, "img or qt is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    const sw::ProjPlan *pp;
    if ((st = get_plan(c, geo.L, geo.n, &pp)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // Fewer images than compute units: one block per image would leave most
    // of the device idle, so project with one block per (image, task group)
    // and invert with 16 waves per image, through scratch.
    const bool small = c->small(N);
    if (!small && sw::tables_fused_fits(geo)) {
        hipError_t e = sw::launch_tables(img, N, geo, *t, *pp, qt, aux, s, c->tables_per_block);
        return e == hipSuccess ? SW_OK : hip_fail(e, "k_tables launch");
    }
    // Otherwise the PMF table of one image does not fit in LDS: project and
    // invert in chunks of images through a bounded scratch buffer.
    const size_t per = sizeof(float) * (size_t)geo.n * geo.L;
    int64_t chunk = (int64_t)((size_t)256 << 20) / (int64_t)per;
    if (chunk < 1) chunk = 1;
    if (chunk > N) chunk = N;
    void *pmf;
    if ((st = get_scratch(c, per * (size_t)chunk, s, &pmf)) != SW_OK) return st;
    for (int64_t i0 = 0; i0 < N; i0 += chunk) {
        const int64_t m = N - i0 < chunk ? N - i0 : chunk;
        hipError_t e = sw::launch_project(img + i0 * (int64_t)geo.L * geo.L, m, geo, *t, *pp,
                                          (float *)pmf, s, small);
        if (e != hipSuccess) return hip_fail(e, "k_project launch");
        e = sw::launch_quantiles((const float *)pmf, m, geo, *t, qt + i0 * (int64_t)geo.Q * geo.n,
                                 aux ? aux + 4 * i0 : nullptr, s, small);
        if (e != hipSuccess) return hip_fail(e, "k_quantile launch");
    }
    return SW_OK;
}

sw_status sw_ramp(void *ctx, const float *pmf, int64_t N, const sw_geom *g, float *out,
                  void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!pmf || !out) return fail(SW_E_INVALID, "pmf or out is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const float *hx;
    if ((st = get_ramp_table(c, geo.L, &hx)) != SW_OK) return st;
    hipError_t e = sw::launch_ramp(pmf, out, N * (int64_t)geo.n, geo.L, hx, (hipStream_t)stream);
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_ramp launch");
}

sw_status sw_quantiles_rf(void *ctx, const float *pf, int64_t N, const sw_geom *g, float *qt,
                          double *aux, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (2 * geo.Q > 512) return fail(SW_E_INVALID, "2 n_quantiles = %d exceeds 512", 2 * geo.Q);
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!pf || !qt) return fail(SW_E_INVALID, "pf or qt is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    hipError_t e = sw::launch_quantiles_rf(pf, N, geo, *t, qt, aux, (hipStream_t)stream,
                                           c->small(N));
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_quantile_rf launch");
}

sw_status sw_tables_rf(void *ctx, const float *img, int64_t N, const sw_geom *g, float *qt,
                       double *aux, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (2 * geo.Q > 512) return fail(SW_E_INVALID, "2 n_quantiles = %d exceeds 512", 2 * geo.Q);
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!img || !qt) return fail(SW_E_INVALID, "img or qt is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    const sw::ProjPlan *pp;
    if ((st = get_plan(c, geo.L, geo.n, &pp)) != SW_OK) return st;
    const float *hx;
    if ((st = get_ramp_table(c, geo.L, &hx)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool small = c->small(N);
    if (!small && sw::tables_rf_fused_fits(geo)) {
        hipError_t e =
            sw::launch_tables_rf(img, N, geo, *t, *pp, hx, qt, aux, s, c->tables_per_block);
        return e == hipSuccess ? SW_OK : hip_fail(e, "k_tables_rf launch");
    }
    // projections of a chunk of images in scratch, filtered in place, then
    // split and inverted
    const size_t per = sizeof(float) * (size_t)geo.n * geo.L;
    int64_t chunk = (int64_t)((size_t)256 << 20) / (int64_t)per;
    if (chunk < 1) chunk = 1;
    if (chunk > N) chunk = N;
    void *pmf;
    if ((st = get_scratch(c, per * (size_t)chunk, s, &pmf)) != SW_OK) return st;
    for (int64_t i0 = 0; i0 < N; i0 += chunk) {
        const int64_t m = N - i0 < chunk ? N - i0 : chunk;
        hipError_t e = sw::launch_project(img + i0 * (int64_t)geo.L * geo.L, m, geo, *t, *pp,
                                          (float *)pmf, s, small);
        if (e != hipSuccess) return hip_fail(e, "k_project launch");
        e = sw::launch_ramp((const float *)pmf, (float *)pmf, m * (int64_t)geo.n, geo.L, hx, s);
        if (e != hipSuccess) return hip_fail(e, "k_ramp launch");
        e = sw::launch_quantiles_rf((const float *)pmf, m, geo, *t,
                                    qt + i0 * (int64_t)2 * geo.Q * geo.n,
                                    aux ? aux + 4 * i0 : nullptr, s, small);
        if (e != hipSuccess) return hip_fail(e, "k_quantile_rf launch");
    }
    return SW_OK;
}

// Geometry and scratch of the Fourier-slice projector: L even with prime
// factors 2 and 3 only (the transforms of lengths L and 2L are mixed-radix
// 4/3/2; powers of two take the shift-indexed kernel).
static sw_status fourier_setup(Ctx *c, const sw::Geo &geo, int64_t N, const double *theta,
                               sw::FourierShape *S, sw::FourierTabs *T, int *slots,
                               const sw::AngleTable **dirs) {
    if (geo.L % 2 != 0 || !only_2_3(geo.L))
        return fail(SW_E_INVALID,
                    "the Fourier-slice projector needs L even with prime factors 2 and 3 only "
                    "(L = %d)",
                    geo.L);
    const int lg = log2_exact(geo.L);  // -1 unless a power of two
    S->L = geo.L;
    S->n = geo.n;
    S->Nf = 2 * geo.L;
    S->lgNf = lg < 0 ? -1 : lg + 1;
    S->lgL = lg;
    S->H = geo.L + 1;
    S->mirror = theta ? 0 : 1;
    sw_status st = get_fourier_tabs(c, geo.L, T);
    if (st != SW_OK) return st;
    if (theta) {
        for (int m = 0; m < geo.n; ++m)
            if (!std::isfinite(theta[m]))
                return fail(SW_E_INVALID, "angle %d is not finite", m);
        st = get_fourier_dir_targets(c, geo.L, geo.n, theta, &T->targets, dirs);
    } else {
        st = get_fourier_targets(c, geo.L, geo.n, &T->targets);
        if (st == SW_OK) st = get_table(c, geo.n, dirs);
    }
    if (st != SW_OK) return st;
    // one slot per block that can be resident at once, at most two per CU (a
    // third block at L = 128 fits but costs 4 % through its scratch traffic)
    const int64_t cap =
        (int64_t)std::min(sw::fourier_blocks_per_cu(S->L, S->Nf), 2) * c->cu_count;
    *slots = (int)(N < cap ? N : cap);
    return SW_OK;
}

static sw_status project_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g,
                                 const double *theta, float *pmf, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!img || !pmf) return fail(SW_E_INVALID, "img or pmf is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    sw::FourierShape S;
    sw::FourierTabs T;
    int slots;
    const sw::AngleTable *dirs;
    if ((st = fourier_setup(c, geo, N, theta, &S, &T, &slots, &dirs)) != SW_OK) return st;
    (void)dirs;  // the projection needs the slice-point table only
    hipStream_t s = (hipStream_t)stream;
    void *scr;
    if ((st = get_scratch(c, sw::fourier_slot_bytes(S.L, S.Nf) * slots, s, &scr)) != SW_OK)
        return st;
    hipError_t e = sw::launch_fourier(img, N, S, T, scr, slots, pmf, s);
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_fourier launch");
}

sw_status sw_project_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g, float *pmf,
                             void *stream) {
    return project_fourier(ctx, img, N, g, nullptr, pmf, stream);
}

sw_status sw_project_fourier_at(void *ctx, const float *img, int64_t N, const sw_geom *g,
                                const double *theta, float *pmf, void *stream) {
    if (!theta) return fail(SW_E_INVALID, "theta is NULL");
    return project_fourier(ctx, img, N, g, theta, pmf, stream);
}

static sw_status tables_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g,
                                const double *theta, float *qt, double *aux, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    sw::Geo geo;
    sw_status st = check_geom(g, &geo);
    if (st != SW_OK) return st;
    if (N < 0) return fail(SW_E_INVALID, "N = %lld is negative", (long long)N);
    if (N == 0) return SW_OK;
    if (!img || !qt) return fail(SW_E_INVALID, "img or qt is NULL");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    sw::FourierShape S;
    sw::FourierTabs T;
    int slots;
    const sw::AngleTable *dirs;
    if ((st = fourier_setup(c, geo, N, theta, &S, &T, &slots, &dirs)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // projections of a chunk of images, then their quantile tables; the
    // scratch holds the chunk's projections and the projector's slots
    const size_t per = sizeof(float) * (size_t)geo.n * geo.L;
    int64_t chunk = (int64_t)((size_t)256 << 20) / (int64_t)per;
    if (chunk < 1) chunk = 1;
    if (chunk > N) chunk = N;
    const size_t pmf_bytes = (per * (size_t)chunk + 255) & ~(size_t)255;
    void *scr;
    if ((st = get_scratch(c, pmf_bytes + sw::fourier_slot_bytes(S.L, S.Nf) * slots, s, &scr)) !=
        SW_OK)
        return st;
    float *pmf = (float *)scr;
    void *slot_mem = (char *)scr + pmf_bytes;
    for (int64_t i0 = 0; i0 < N; i0 += chunk) {
        const int64_t m = N - i0 < chunk ? N - i0 : chunk;
        hipError_t e = sw::launch_fourier(img + i0 * (int64_t)geo.L * geo.L, m, S, T, slot_mem,
                                          slots, pmf, s);
        if (e != hipSuccess) return hip_fail(e, "k_fourier launch");
        e = sw::launch_quantiles(pmf, m, geo, *dirs, qt + i0 * (int64_t)geo.Q * geo.n,
                                 aux ? aux + 4 * i0 : nullptr, s, c->small(m));
        if (e != hipSuccess) return hip_fail(e, "k_quantile launch");
    }
    return SW_OK;
}

sw_status sw_tables_fourier(void *ctx, const float *img, int64_t N, const sw_geom *g, float *qt,
                            double *aux, void *stream) {
    return tables_fourier(ctx, img, N, g, nullptr, qt, aux, stream);
}

sw_status sw_tables_fourier_at(void *ctx, const float *img, int64_t N, const sw_geom *g,
                               const double *theta, float *qt, double *aux, void *stream) {
    if (!theta) return fail(SW_E_INVALID, "theta is NULL");
    return tables_fourier(ctx, img, N, g, theta, qt, aux, stream);
}

// sw_align_batch and sw_align_batch_noalloc: with noalloc the angle table
// and the scratch come from the file-scope array of the device, and a call
// needing more scratch than it holds fails.
static sw_status align_batch_impl(void *ctx, const sw_batch *b, sw_result *out, float *curve,
                                  void *stream, bool noalloc) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    if (!b) return fail(SW_E_INVALID, "batch is NULL");
    sw::Geo geo;
    sw_status st = check_geom(&b->geom, &geo);
    if (st != SW_OK) return st;
    if (b->filter != SW_FILTER_NONE && b->filter != SW_FILTER_RAMP)
        return fail(SW_E_INVALID, "filter = %d is not a sw_filter value", b->filter);
    const bool ramp = b->filter == SW_FILTER_RAMP;
    if (ramp) {
        // the stacked tables align as one table of 2Q rows; the distance of
        // the two parts is twice that table's objective
        if (2 * geo.Q > 512) return fail(SW_E_INVALID, "2 n_quantiles = %d exceeds 512", 2 * geo.Q);
        geo.Q *= 2;
    }
    if (b->n_ref < 0 || b->n_img < 0 || b->n_pairs < 0)
        return fail(SW_E_INVALID, "negative count");
    const int64_t P = b->pairs ? b->n_pairs : b->n_ref * b->n_img;
    if (P == 0) return SW_OK;
    if (!b->ref_qt || !b->ref_aux || !b->img_qt || !b->img_aux || !out)
        return fail(SW_E_INVALID, "a table, aux or output pointer is NULL");
    if (b->n_ref == 0 || b->n_img == 0)
        return fail(SW_E_INVALID, "pairs given but a table set is empty");
    if (b->mode != SW_MODE_ROT_TRANS && b->mode != SW_MODE_ROT_ONLY &&
        b->mode != SW_MODE_MAX_SLICED)
        return fail(SW_E_INVALID, "mode = %d is not a sw_mode value", b->mode);
    if (b->mode == SW_MODE_MAX_SLICED && !sw::msw_supported(geo))
        return fail(SW_E_UNSUPPORTED,
                    "max-sliced alignment needs n_angles a multiple of 16 up to 128, got %d",
                    geo.n);
    if (b->prec != SW_PREC_FP32 && b->prec != SW_PREC_BF16_SPLIT)
        return fail(SW_E_INVALID, "prec = %d is not a sw_precision value", b->prec);
    int top_k = b->top_k;
    if (top_k == 0) top_k = b->prec == SW_PREC_BF16_SPLIT ? 4 : 1;
    if (top_k < 1 || top_k > sw::kMaxTopK || top_k > geo.n)
        return fail(SW_E_INVALID, "top_k = %d outside [1, min(%d, n)]", b->top_k, sw::kMaxTopK);
    if (P > 0x7fffffffLL) return fail(SW_E_INVALID, "too many pairs in one call (%lld)", (long long)P);
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    const sw::AngleTable *t;
    NoAllocDevice *na = nullptr;
    if (noalloc) {
        if ((st = noalloc_device(c->device, &na)) != SW_OK) return st;
        t = &na->tables.at(geo.n);  // every admissible n is there
    } else if ((st = get_table(c, geo.n, &t)) != SW_OK) {
        return st;
    }
    // the call's scratch: the context's (grown on demand) or the array's
    auto take_scratch = [&](size_t bytes, void **p) -> sw_status {
        if (!noalloc) return get_scratch(c, bytes, (hipStream_t)stream, p);
        if (bytes > kNoAllocWorkBytes)
            return fail(SW_E_NOMEM,
                        "the call needs %zu bytes of scratch; sw_align_batch_noalloc holds %zu",
                        bytes, kNoAllocWorkBytes);
        *p = na->work;
        return SW_OK;
    };
    hipStream_t s = (hipStream_t)stream;
    if (b->mode == SW_MODE_MAX_SLICED) {
        sw::PairArgs a{};
        a.ref_qt = b->ref_qt;
        a.ref_aux = b->ref_aux;
        a.n_ref = b->n_ref;
        a.img_qt = b->img_qt;
        a.img_aux = b->img_aux;
        a.n_img = b->n_img;
        a.pairs = b->pairs;
        a.n_pairs = b->n_pairs;
        a.mode = b->mode;
        a.top_k = top_k;
        a.out = (sw::Result *)out;
        a.curve = curve;
        hipError_t e = sw::launch_align_msw(a, geo, s);
        if (e != hipSuccess) return hip_fail(e, "k_align_msw launch");
        if (ramp) {
            e = sw::launch_scale_results((sw::Result *)out, P, curve, geo.n, 2.f, s);
            if (e != hipSuccess) return hip_fail(e, "k_scale_results launch");
        }
        return SW_OK;
    }
    const int Wn = geo.n / 2 + 1;
    const bool same_set = b->ref_qt == b->img_qt && b->ref_aux == b->img_aux && b->n_ref == b->n_img;
    if (!b->pairs && !curve && b->prec == SW_PREC_BF16_SPLIT && top_k <= 4 &&
        sw::mfma_path_supported(geo) && P >= 256) {
        // many-vs-many on the matrix cores: bf16 spectra of both sets, then
        // the correlation/top-k kernel and the FP32 rescore
        const size_t per = sizeof(uint32_t) * (size_t)Wn * geo.Q;
        const size_t ref_bytes = (per * (size_t)b->n_ref + 255) & ~(size_t)255;
        const size_t img_bytes = same_set ? 0 : (per * (size_t)b->n_img + 255) & ~(size_t)255;
        const size_t cand_bytes = sizeof(int16_t) * (size_t)P * top_k;
        void *scr;
        if ((st = take_scratch(ref_bytes + img_bytes + cand_bytes, &scr)) != SW_OK) return st;
        char *base = (char *)scr;
        uint32_t *spec_ref = (uint32_t *)base;
        uint32_t *spec_img = same_set ? spec_ref : (uint32_t *)(base + ref_bytes);
        int16_t *cand = (int16_t *)(base + ref_bytes + img_bytes);
        hipError_t e = sw::launch_spectrum(b->ref_qt, b->n_ref, geo, *t, spec_ref, 1, s);
        if (e == hipSuccess && !same_set)
            e = sw::launch_spectrum(b->img_qt, b->n_img, geo, *t, spec_img, 1, s);
        if (e != hipSuccess) return hip_fail(e, "k_spectrum launch");
        sw::MfmaArgs m;
        m.spec_ref = spec_ref;
        m.spec_img = spec_img;
        m.ref_qt = b->ref_qt;
        m.ref_aux = b->ref_aux;
        m.n_ref = b->n_ref;
        m.img_qt = b->img_qt;
        m.img_aux = b->img_aux;
        m.n_img = b->n_img;
        m.mode = b->mode;
        m.top_k = top_k;
        m.cand = cand;
        m.out = (sw::Result *)out;
        e = sw::launch_mfma_all_pairs(m, geo, *t, s);
        if (e != hipSuccess) return hip_fail(e, "k_corr_mfma / k_rescore_tiles launch");
        if (ramp) {
            e = sw::launch_scale_results((sw::Result *)out, P, nullptr, geo.n, 2.f, s);
            if (e != hipSuccess) return hip_fail(e, "k_scale_results launch");
        }
        return SW_OK;
    }
    const size_t spec_bytes =
        (sizeof(float2) * (size_t)Wn * geo.Q * (size_t)b->n_ref + 255) & ~(size_t)255;
    const bool fast128 = sw::align128_supported(geo) && !c->generic_align;
    const size_t gam_bytes = fast128 ? sw::align128_scratch_bytes(geo, b->n_ref) : 0;
    void *spec;
    if ((st = take_scratch(spec_bytes + gam_bytes, &spec)) != SW_OK) return st;
    hipError_t e = sw::launch_spectrum(b->ref_qt, b->n_ref, geo, *t, spec, 0, s);
    if (e != hipSuccess) return hip_fail(e, "k_spectrum launch");
    sw::PairArgs a;
    a.ref_qt = b->ref_qt;
    a.ref_aux = b->ref_aux;
    a.ref_spec = (const float2 *)spec;
    a.n_ref = b->n_ref;
    a.img_qt = b->img_qt;
    a.img_aux = b->img_aux;
    a.n_img = b->n_img;
    a.pairs = b->pairs;
    a.n_pairs = b->n_pairs;
    a.mode = b->mode;
    a.bf16 = b->prec == SW_PREC_BF16_SPLIT;
    a.top_k = top_k;
    a.out = (sw::Result *)out;
    a.curve = curve;
    if (fast128) {
        e = sw::launch_align128(a, geo, *t, (float2 *)((char *)spec + spec_bytes), s,
                                c->align128_per_wave);
        if (e != hipSuccess) return hip_fail(e, "k_gamma128 / k_align128 launch");
    } else {
        e = sw::launch_align_pairs(a, geo, *t, s);
        if (e != hipSuccess) return hip_fail(e, "k_align_pairs launch");
    }
    if (ramp) {
        e = sw::launch_scale_results((sw::Result *)out, P, curve, geo.n, 2.f, s);
        if (e != hipSuccess) return hip_fail(e, "k_scale_results launch");
    }
    return SW_OK;
}

sw_status sw_align_batch(void *ctx, const sw_batch *b, sw_result *out, float *curve,
                         void *stream) {
    return align_batch_impl(ctx, b, out, curve, stream, false);
}

sw_status sw_align_batch_noalloc(void *ctx, const sw_batch *b, sw_result *out, float *curve,
                                 void *stream) {
    return align_batch_impl(ctx, b, out, curve, stream, true);
}

sw_status sw_align_stacks(void *ctx, const sw_stack *stacks, int32_t n_stacks, int32_t mode,
                          int32_t prec, int32_t top_k, void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    if (n_stacks < 0 || (n_stacks > 0 && !stacks)) return fail(SW_E_INVALID, "bad stack list");
    if (mode != SW_MODE_ROT_TRANS && mode != SW_MODE_ROT_ONLY)
        return fail(SW_E_INVALID, "mode = %d is not a sw_mode value", mode);
    if (prec != SW_PREC_FP32 && prec != SW_PREC_BF16_SPLIT)
        return fail(SW_E_INVALID, "prec = %d is not a sw_precision value", prec);
    if (top_k == 0) top_k = prec == SW_PREC_BF16_SPLIT ? 4 : 1;
    if (top_k < 1 || top_k > sw::kMaxTopK) return fail(SW_E_INVALID, "top_k = %d", top_k);
    std::vector<const sw_stack *> live;
    for (int i = 0; i < n_stacks; ++i) {
        const sw_stack &k = stacks[i];
        sw::Geo geo;
        sw_status st = check_geom(&k.geom, &geo);
        if (st != SW_OK) return fail(st, "stack %d: %s", i, g_err.c_str());
        if (k.N < 0) return fail(SW_E_INVALID, "stack %d: N < 0", i);
        if (top_k > geo.n) return fail(SW_E_INVALID, "stack %d: top_k > n", i);
        if (k.N == 0) continue;
        if (!k.ref_img || !k.imgs || !k.ref_qt || !k.ref_aux || !k.qt || !k.aux || !k.out)
            return fail(SW_E_INVALID, "stack %d: a pointer is NULL", i);
        live.push_back(&k);
    }
    if (live.empty()) return SW_OK;
    // largest images first so that the tail of the work queue is short
    std::stable_sort(live.begin(), live.end(), [](const sw_stack *a, const sw_stack *b) {
        return a->geom.L > b->geom.L;
    });
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    for (size_t i0 = 0; i0 < live.size(); i0 += sw::kMaxMix) {
        const int m = (int)std::min(live.size() - i0, (size_t)sw::kMaxMix);
        sw_status st = run_stack_chunk(c, live.data() + i0, m, mode, prec == SW_PREC_BF16_SPLIT,
                                       top_k, 0, (hipStream_t)stream);
        if (st != SW_OK) return st;
    }
    return SW_OK;
}

sw_status sw_autotune(void *ctx, const int32_t *Ls, int32_t nL, int64_t n_images,
                      const char *out_json) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    if (nL < 0 || (nL > 0 && !Ls)) return fail(SW_E_INVALID, "bad L list");
    if (n_images < 1 || n_images > (1 << 20)) return fail(SW_E_INVALID, "n_images out of range");
    Ctx *c = as_ctx(ctx);
    DeviceGuard dg(c->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    std::map<int, int> best_R, best_tpw, best_bpc;  // 0: the default
    std::map<int, float> best_ms;
    for (int li = 0; li < nL; ++li) {
        const int L = Ls[li];
        sw_geom g{L, L, L, SW_LEVELS_MIDPOINT};
        sw::Geo geo;
        sw_status st = check_geom(&g, &geo);
        if (st != SW_OK) return st;
        const size_t nimg = (size_t)n_images * L * L, ntab = (size_t)n_images * L * L;
        float *img = nullptr, *qt = nullptr, *rqt = nullptr;
        double *aux = nullptr, *raux = nullptr;
        sw_result *out = nullptr;
        hipError_t e = hipMalloc(&img, sizeof(float) * nimg);
        if (e == hipSuccess) e = hipMalloc(&qt, sizeof(float) * ntab);
        if (e == hipSuccess) e = hipMalloc(&rqt, sizeof(float) * L * L);
        if (e == hipSuccess) e = hipMalloc(&aux, sizeof(double) * 4 * n_images);
        if (e == hipSuccess) e = hipMalloc(&raux, sizeof(double) * 4);
        if (e == hipSuccess) e = hipMalloc(&out, sizeof(sw_result) * n_images);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = sw::launch_fill_synthetic(img, (int64_t)nimg, nullptr);
        sw_stack k{img, img, (int64_t)n_images, g, rqt, raux, qt, aux, out};
        const sw_stack *kp = &k;
        // time one configuration: best of three runs after a warm-up
        auto measure = [&](int R, const sw::MixKnobs &kn) -> float {
            float tbest = 1e30f;
            for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, nullptr);
                if (e == hipSuccess) {
                    st = run_stack_chunk(c, &kp, 1, SW_MODE_ROT_TRANS, 0, 1, R, nullptr, &kn);
                    if (st != SW_OK) e = hipErrorUnknown;
                }
                if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0 && ms < tbest) tbest = ms;  // the first run warms up
            }
            return tbest;
        };
        // coordinate descent: strip rows, then tasks per wave of the tables
        // kernel, then blocks per compute unit of the per-pair alignment
        sw::MixKnobs kn;
        const int Rmax = sw::strip4_rows_max(L);
        int bR = 0;
        float bms = 1e30f;
        const int cands[] = {2, 4, 6, 8, 12, 16, 24, 32, 0};  // 0: the largest that fits
        for (int R : cands) {
            if (e != hipSuccess) break;
            if (R == 0) R = Rmax;
            else if (R >= Rmax) continue;
            const float ms = measure(R, kn);
            if (e == hipSuccess && ms < bms) {
                bms = ms;
                bR = R;
            }
        }
        int btpw = 0;
        for (int tpw : {sw::kMixTablesTasksSmall, sw::kMixTablesTasks, sw::kMixTablesTasksLarge}) {
            if (e != hipSuccess) break;
            sw::MixKnobs k2 = kn;
            k2.tpw = tpw;
            const float ms = measure(bR, k2);
            if (e == hipSuccess && ms < bms) {
                bms = ms;
                btpw = tpw;
            }
        }
        kn.tpw = btpw;
        int bbpc = 0;
        for (int bpc : {2, 4, 6, 8}) {
            if (e != hipSuccess) break;
            sw::MixKnobs k2 = kn;
            k2.align_bpc = bpc;
            const float ms = measure(bR, k2);
            if (e == hipSuccess && ms < bms) {
                bms = ms;
                bbpc = bpc;
            }
        }
        if (e == hipSuccess) {
            best_R[L] = bR;
            best_ms[L] = bms;
            best_tpw[L] = btpw;
            best_bpc[L] = bbpc;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(img);
        (void)hipFree(qt);
        (void)hipFree(rqt);
        (void)hipFree(aux);
        (void)hipFree(raux);
        (void)hipFree(out);
        if (e != hipSuccess) return hip_fail(e, "autotune run");
    }
    for (auto &kv : best_R) {
        const int L = kv.first;
        c->tile_R[L] = kv.second;
        if (best_tpw[L]) c->tile_tpw[L] = best_tpw[L];
        else c->tile_tpw.erase(L);
        if (best_bpc[L]) c->tile_abpc[L] = best_bpc[L];
        else c->tile_abpc.erase(L);
    }
    if (out_json && *out_json) {
        std::ofstream f(out_json);
        if (!f) return fail(SW_E_INVALID, "cannot write %s", out_json);
        f << "{\"tiles\": {";
        bool firstk = true;
        for (auto &kv : best_R) {
            const int L = kv.first;
            f << (firstk ? "" : ", ") << "\"" << L << "\": {\"R\": " << kv.second;
            if (best_tpw[L]) f << ", \"tpw\": " << best_tpw[L];
            if (best_bpc[L]) f << ", \"align_bpc\": " << best_bpc[L];
            f << ", \"ms\": " << best_ms[L] << ", \"images\": " << n_images << "}";
            firstk = false;
        }
        f << "}}\n";
    }
    return SW_OK;
}

}  // extern "C"
