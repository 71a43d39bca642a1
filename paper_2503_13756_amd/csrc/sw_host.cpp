// Host runtime of libswalign: contexts, geometry checks, angle tables,
// scratch, and the C entry points declared in include/swalign.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "swalign.h"
#include "sw_internal.h"

namespace {

thread_local std::string g_err;

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

struct Ctx {
    int device = 0;
    std::mutex mu;
    std::map<int, sw::AngleTable> tables;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

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

Ctx *as_ctx(void *p) { return static_cast<Ctx *>(p); }

}  // namespace

extern "C" {

const char *sw_last_error(void) { return g_err.c_str(); }

const char *sw_version(void) { return "swalign 0.1 (gfx950)"; }

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
    *ctx = c;
    return SW_OK;
}

sw_status sw_ctx_destroy(void *ctx) {
    if (!ctx) return SW_OK;
    Ctx *c = as_ctx(ctx);
    {
        DeviceGuard dg(c->device);
        (void)hipDeviceSynchronize();
        for (auto &kv : c->tables) {
            (void)hipFree(kv.second.d32);
            (void)hipFree(kv.second.d64);
        }
        if (c->scratch) (void)hipFree(c->scratch);
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
    hipError_t e = sw::launch_project(img, N, geo, *t, pmf, (hipStream_t)stream);
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
    hipError_t e = sw::launch_quantiles(pmf, N, geo, *t, qt, aux, (hipStream_t)stream);
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
    hipStream_t s = (hipStream_t)stream;
    if (sw::tables_fused_fits(geo)) {
        hipError_t e = sw::launch_tables(img, N, geo, *t, qt, aux, s);
        return e == hipSuccess ? SW_OK : hip_fail(e, "k_tables launch");
    }
    // The PMF table of one image does not fit in LDS: project and invert in
    // chunks of images through a bounded scratch buffer.
    const size_t per = sizeof(float) * (size_t)geo.n * geo.L;
    int64_t chunk = (int64_t)((size_t)256 << 20) / (int64_t)per;
    if (chunk < 1) chunk = 1;
    if (chunk > N) chunk = N;
    void *pmf;
    if ((st = get_scratch(c, per * (size_t)chunk, s, &pmf)) != SW_OK) return st;
    for (int64_t i0 = 0; i0 < N; i0 += chunk) {
        const int64_t m = N - i0 < chunk ? N - i0 : chunk;
        hipError_t e = sw::launch_project(img + i0 * (int64_t)geo.L * geo.L, m, geo, *t,
                                          (float *)pmf, s);
        if (e != hipSuccess) return hip_fail(e, "k_project launch");
        e = sw::launch_quantiles((const float *)pmf, m, geo, *t, qt + i0 * (int64_t)geo.Q * geo.n,
                                 aux ? aux + 4 * i0 : nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "k_quantile launch");
    }
    return SW_OK;
}

sw_status sw_align_batch(void *ctx, const sw_batch *b, sw_result *out, float *curve,
                         void *stream) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    if (!b) return fail(SW_E_INVALID, "batch is NULL");
    sw::Geo geo;
    sw_status st = check_geom(&b->geom, &geo);
    if (st != SW_OK) return st;
    if (b->n_ref < 0 || b->n_img < 0 || b->n_pairs < 0)
        return fail(SW_E_INVALID, "negative count");
    const int64_t P = b->pairs ? b->n_pairs : b->n_ref * b->n_img;
    if (P == 0) return SW_OK;
    if (!b->ref_qt || !b->ref_aux || !b->img_qt || !b->img_aux || !out)
        return fail(SW_E_INVALID, "a table, aux or output pointer is NULL");
    if (b->n_ref == 0 || b->n_img == 0)
        return fail(SW_E_INVALID, "pairs given but a table set is empty");
    if (b->mode != SW_MODE_ROT_TRANS && b->mode != SW_MODE_ROT_ONLY)
        return fail(SW_E_INVALID, "mode = %d is not a sw_mode value", b->mode);
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
    if ((st = get_table(c, geo.n, &t)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
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
        if ((st = get_scratch(c, ref_bytes + img_bytes + cand_bytes, s, &scr)) != SW_OK) return st;
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
        return e == hipSuccess ? SW_OK : hip_fail(e, "k_corr_mfma / k_rescore_tiles launch");
    }
    const size_t spec_bytes = sizeof(float2) * (size_t)Wn * geo.Q * (size_t)b->n_ref;
    void *spec;
    if ((st = get_scratch(c, spec_bytes, s, &spec)) != SW_OK) return st;
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
    e = sw::launch_align_pairs(a, geo, *t, s);
    return e == hipSuccess ? SW_OK : hip_fail(e, "k_align_pairs launch");
}

}  // extern "C"
