// Host-side internals of libswalign shared by the C entry points
// (sw_host.cpp) and the serving runtime (sw_serve.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "swalign.h"
#include "fourier_internal.h"
#include "mix_internal.h"
#include "sw_internal.h"

namespace swh {

sw_status fail(sw_status s, const char *fmt, ...);
sw_status hip_fail(hipError_t e, const char *where);
const std::string &last_error();

// Pinned host staging of the device-side stack descriptors: a ring of slots,
// each reused only after the copy that last read it has completed.
struct DescRing {
    static constexpr int kSlots = 8;
    sw::MixGroup *host = nullptr;  // [kSlots][2]
    hipEvent_t ev[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
};

struct Server;  // serving runtime (sw_serve.cpp)

struct Ctx {
    int device = 0;
    int cu_count = 256;
    std::mutex mu;
    std::map<int, sw::AngleTable> tables;
    std::map<int, sw::ProjPlan> plans;  // key L * 4096 + n
    std::map<int, float *> ramp_tables;  // ramp filter kernel per L
    std::map<int, void *> fourier_tabs;     // Fourier-slice projector tables per L
    std::map<int, void *> fourier_targets;  // its slice-point tables, key L * 4096 + n
    // slice-point tables for explicit angles: (L, n, the angles' bytes) -> table
    std::map<std::string, void *> fourier_dir_targets;
    std::map<std::string, sw::AngleTable> fourier_dir_angles;  // their direction tables
    std::map<int, int> tile_R;     // projection strip rows per L (autotuner)
    std::map<int, int> tile_tpw;   // tables kernel tasks per wave per L (autotuner)
    std::map<int, int> tile_abpc;  // alignment blocks per compute unit per L (autotuner)
    // the launch knobs of a mixed launch: those tuned for the L with the most
    // projection work (images x L^3) among the given (L, images) pairs
    sw::MixKnobs knobs_for(const std::vector<std::pair<int, int64_t>> &items) const {
        sw::MixKnobs k;
        int best = -1;
        double work = -1.0;
        for (auto &it : items) {
            const double w = (double)it.second * it.first * it.first * it.first;
            if (w > work) {
                work = w;
                best = it.first;
            }
        }
        auto a = tile_tpw.find(best), b = tile_abpc.find(best);
        if (a != tile_tpw.end()) k.tpw = a->second;
        if (b != tile_abpc.end()) k.align_bpc = b->second;
        return k;
    }
    // batches of fewer images take the split (many blocks per image) launches;
    // -1: the number of compute units
    int small_batch = -1;
    bool generic_align = false;  // never use the n = 128 register-FFT kernel
    bool align128_per_wave = true;  // n = 128: one pair per wave (else per block)
    int tables_per_block = 2;    // images per block of the fused tables kernel (1 or 2)
    // failure injection for tests of the serving runtime: the request with
    // this ticket has its host-to-device copy reported as failed (0: none)
    uint64_t serve_fail_ticket = 0;
    bool small(int64_t N) const { return N < (small_batch >= 0 ? small_batch : cu_count); }
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    DescRing ring;
    Server *server = nullptr;
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

sw_status check_geom(const sw_geom *g, sw::Geo *out);
sw_status get_table(Ctx *ctx, int n, const sw::AngleTable **out);
sw_status get_plan(Ctx *ctx, int L, int n, const sw::ProjPlan **out);
void stop_server(Ctx *c);

}  // namespace swh
