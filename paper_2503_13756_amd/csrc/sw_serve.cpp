// Serving runtime of libswalign: continuous batching of alignment requests.
//
// A scheduler thread per context admits requests from a FIFO queue while
// they fit in a first-fit HBM arena and a slot is free, copies their images
// on a copy stream, and issues "steps" on a compute stream: every admitted
// request of one geometry (up to max_per_step) goes into one sequence of mixed
// persistent kernels (reference tables, reference spectra, image tables,
// alignment).  The sequence is captured once per geometry as a hipGraph and
// replayed; each replay reads new descriptor contents that were copied into a
// fixed device buffer just before it on the same stream.  Steps are issued
// without waiting for the previous one, so the device queue stays full while
// the host admits the next requests.  Completion is tracked with one event
// per step; results land in pinned host buffers and are handed out by poll.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_internal.h"

namespace swh {

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        free_[0] = size;
        size_ = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

enum class RState { Pending, Admitted, Launched, Done, Cancelled, Failed };

// A cached reference table.  Its tables are usable once the step of the
// request that computes them (the producer) has completed without error;
// until then only requests in that step or in later steps on the same
// stream may read them.  A producer that fails before or during its step
// leaves the entry without a producer: the next request of that key to be
// launched computes the tables itself, and requests that were launched
// behind the failed producer (gen changed since their launch) fail.
struct RefEntry {
    uint64_t key = 0;
    size_t off = 0, bytes = 0;
    int L = 0, n = 0, Q = 0, levels = 0;
    int users = 0;
    uint64_t last_use = 0;
    bool ready = false;     // written by a step that completed without error
    uint64_t producer = 0;  // ticket of the request whose step writes it (0: none)
    uint64_t gen = 0;       // bumped whenever a producer fails
};

struct Step {
    hipEvent_t done = nullptr;
    std::vector<uint64_t> tickets;
};

// Pinned host buffers for results, reused across requests in power-of-two
// size classes: pinned allocation and release stay off the request path
// (releasing pinned memory can wait for the device to drain).  Guarded by
// the server mutex; everything is released when serving stops.
class PinPool {
  public:
    void *get(size_t bytes, size_t *cap) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        *cap = c;
        auto it = free_.find(c);
        if (it != free_.end()) {
            void *p = it->second;
            free_.erase(it);
            return p;
        }
        void *p = nullptr;
        return hipHostMalloc(&p, c) == hipSuccess ? p : nullptr;
    }
    void put(void *p, size_t cap) {
        if (p) free_.emplace(cap, p);
    }
    void clear() {
        for (auto &kv : free_) (void)hipHostFree(kv.second);
        free_.clear();
    }

  private:
    std::multimap<size_t, void *> free_;
};

struct Req {
    uint64_t ticket = 0;
    sw_request r{};
    sw::Geo geo{};
    RState state = RState::Pending;
    bool cancel = false;
    size_t off = 0, bytes = 0;  // own arena region
    size_t o_img = 0, o_ref = 0, o_qt = 0, o_aux = 0, o_out = 0, o_spec = 0, o_gam = 0,
           o_rqt = 0, o_raux = 0;  // absolute arena offsets
    uint64_t ref_key = 0;       // cache entry used (0 = own tables)
    bool ref_compute = false;   // this request's step computes the reference tables
    uint64_t ref_gen = 0;       // generation of the cache entry at launch
    bool waited_memory = false, waited_slot = false;  // held at the head of the queue
    sw_result *host_out = nullptr;
    size_t host_cap = 0;  // size class of host_out in the pin pool
    hipEvent_t copied = nullptr;
    std::string err;
};

}  // namespace

struct Server {
    sw_serve_cfg cfg{};
    Ctx *ctx = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    Arena arena;
    char *base = nullptr;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> admitted;  // admitted, not launched (arrival order)
    std::deque<Step> steps;          // launched, not finished
    std::unordered_map<uint64_t, RefEntry> cache;
    uint64_t clock = 0, next_ticket = 1;
    sw_serve_stats st{};
    hipStream_t copy_s = nullptr, comp_s = nullptr;
    sw::MixGroup *d_groups = nullptr;     // [2] live descriptors
    unsigned long long *d_cnt = nullptr;  // [4]
    float *d_slots = nullptr;             // grid PMF slots
    int64_t slot_floats = 0;
    int grid = 512;
    std::map<std::vector<int>, hipGraphExec_t> graphs;
    DescRing ring;  // pinned descriptor staging of this server
    PinPool pins;   // pinned result buffers
};

namespace {

sw_status require_server(Ctx *c, Server **s) {
    if (!c) return fail(SW_E_INVALID, "ctx is NULL");
    if (!c->server) return fail(SW_E_INVALID, "serving is not started on this context");
    *s = c->server;
    return SW_OK;
}

// register-FFT coefficients of the reference (n = 128 only)
size_t gam_bytes(const sw::Geo &g) {
    return sw::align128_supported(g) ? sw::align128_scratch_bytes(g, 1) : 0;
}

size_t request_bytes(const sw_request &r, const sw::Geo &g, bool own_ref_tables) {
    const size_t N = (size_t)r.N, L2 = (size_t)g.L * g.L, T = (size_t)g.Q * g.n;
    size_t b = up(4 * N * L2) + up(4 * N * T) + up(32 * N) + up(24 * N) + up(4 * L2) +
               up(8 * (size_t)(g.n / 2 + 1) * g.Q) + up(gam_bytes(g));
    if (own_ref_tables) b += up(4 * T) + up(32);
    return b;
}

// Free arena memory by evicting an unused cached reference table (LRU).
bool evict_one(Server *s) {
    auto victim = s->cache.end();
    for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
        if (it->second.users == 0 &&
            (victim == s->cache.end() || it->second.last_use < victim->second.last_use))
            victim = it;
    if (victim == s->cache.end()) return false;
    s->arena.release(victim->second.off, victim->second.bytes);
    s->cache.erase(victim);
    ++s->st.evictions;
    return true;
}

bool alloc_evicting(Server *s, size_t bytes, size_t *off) {
    while (!s->arena.alloc(bytes, off))
        if (!evict_one(s)) return false;
    return true;
}

// Admission (lock held): FIFO, while slots and memory allow.
void admit(Server *s, std::vector<Req *> &fresh) {
    int64_t live = (int64_t)s->admitted.size();
    for (auto &stp : s->steps) live += (int64_t)stp.tickets.size();
    for (;;) {
        if (s->pending.empty()) break;
        if (live >= s->cfg.max_slots) {
            s->reqs[s->pending.front()]->waited_slot = true;
            break;
        }
        Req *q = s->reqs[s->pending.front()].get();
        const sw::Geo &g = q->geo;
        const uint64_t key = q->r.ref_key;
        auto ce = key ? s->cache.find(key) : s->cache.end();
        const bool cached = ce != s->cache.end() && ce->second.L == g.L && ce->second.n == g.n &&
                            ce->second.Q == g.Q && ce->second.levels == g.levels;
        if (key && ce != s->cache.end() && !cached) {
            // same key, other geometry: the old entry is replaced once unused
            if (ce->second.users > 0) break;
            s->arena.release(ce->second.off, ce->second.bytes);
            s->cache.erase(ce);
        }
        const bool own_ref = key == 0;
        size_t off = 0, need = request_bytes(q->r, g, own_ref);
        size_t ref_off = 0, ref_bytes = up(4 * (size_t)g.Q * g.n) + up(32);
        if (key && !cached) {
            if (!alloc_evicting(s, ref_bytes, &ref_off)) {
                q->waited_memory = true;
                break;
            }
        }
        if (!alloc_evicting(s, need, &off)) {
            if (key && !cached) s->arena.release(ref_off, ref_bytes);
            q->waited_memory = true;
            break;
        }
        if (key && !cached) {
            RefEntry e;
            e.key = key;
            e.off = ref_off;
            e.bytes = ref_bytes;
            e.L = g.L;
            e.n = g.n;
            e.Q = g.Q;
            e.levels = g.levels;
            e.producer = q->ticket;
            s->cache[key] = e;
            q->ref_compute = true;
        } else if (cached) {
            ++s->st.cache_hits;
            q->ref_compute = false;
        } else {
            q->ref_compute = true;
        }
        q->off = off;
        q->bytes = need;
        const size_t N = (size_t)q->r.N, L2 = (size_t)g.L * g.L, T = (size_t)g.Q * g.n;
        size_t o = off;
        q->o_img = o;
        o += up(4 * N * L2);
        q->o_qt = o;
        o += up(4 * N * T);
        q->o_aux = o;
        o += up(32 * N);
        q->o_out = o;
        o += up(24 * N);
        q->o_ref = o;
        o += up(4 * L2);
        q->o_spec = o;
        o += up(8 * (size_t)(g.n / 2 + 1) * g.Q);
        q->o_gam = o;
        o += up(gam_bytes(g));
        if (own_ref) {
            q->o_rqt = o;
            o += up(4 * T);
            q->o_raux = o;
            q->ref_key = 0;
        } else {
            RefEntry &e = s->cache[key];
            q->o_rqt = e.off;
            q->o_raux = e.off + up(4 * T);
            q->ref_key = key;
            ++e.users;
            e.last_use = ++s->clock;
        }
        q->host_out = (sw_result *)s->pins.get(sizeof(sw_result) * (size_t)q->r.N, &q->host_cap);
        if (!q->host_out) q->err = "hipHostMalloc for the results failed";
        q->state = RState::Admitted;
        s->pending.pop_front();
        s->admitted.push_back(q->ticket);
        fresh.push_back(q);
        ++s->st.admitted;
        s->st.waited_memory += q->waited_memory;
        s->st.waited_slot += q->waited_slot;
        ++live;
    }
}

// A request that computes cached reference tables has failed (before or in
// its step): the entry loses its producer, and requests launched behind it
// are failed by the generation check at their completion.
void producer_failed(Server *s, Req *q) {
    if (!q->ref_key || !q->ref_compute) return;
    auto it = s->cache.find(q->ref_key);
    if (it == s->cache.end() || it->second.producer != q->ticket) return;
    it->second.producer = 0;
    it->second.ready = false;
    ++it->second.gen;
}

// Before a step is issued (lock held): every request of the batch that reads
// a cached reference table whose tables are neither ready nor being computed
// by this batch or by a step in flight computes them itself.
void assign_producers(Server *s, const std::vector<Req *> &batch) {
    for (Req *q : batch) {
        if (!q->ref_key) continue;
        auto ce = s->cache.find(q->ref_key);
        if (ce == s->cache.end()) continue;  // cannot happen while q uses it
        RefEntry &e = ce->second;
        if (q->ref_compute) {
            e.producer = q->ticket;
        } else if (!e.ready) {
            bool alive = false;
            for (Req *o : batch) alive |= o->ticket == e.producer && o->ref_compute;
            if (!alive && e.producer) {
                auto it = s->reqs.find(e.producer);
                alive = it != s->reqs.end() && it->second->state == RState::Launched;
            }
            if (!alive) {
                q->ref_compute = true;
                e.producer = q->ticket;
            }
        }
        q->ref_gen = e.gen;
    }
}

// At the completion of a step without error (lock held): false when the
// request read reference tables whose producer failed after it was launched.
bool reference_ok(Server *s, Req *q) {
    if (!q->ref_key) return true;
    auto it = s->cache.find(q->ref_key);
    if (it == s->cache.end()) return true;
    RefEntry &e = it->second;
    if (q->ref_compute && e.producer == q->ticket) {
        e.ready = true;
        e.producer = 0;
        return true;
    }
    return q->ref_compute || e.gen == q->ref_gen;
}

void release_request(Server *s, Req *q) {
    if (q->bytes) s->arena.release(q->off, q->bytes);
    q->bytes = 0;
    if (q->ref_key) {
        auto it = s->cache.find(q->ref_key);
        if (it != s->cache.end() && it->second.users > 0) --it->second.users;
    }
    if (q->copied) {
        (void)hipEventDestroy(q->copied);
        q->copied = nullptr;
    }
}

// Build and issue one step for the given requests (same geometry).  Runs on
// the scheduler thread without the lock; requests are owned by it here.
hipError_t issue_step(Server *s, const std::vector<Req *> &rs, hipEvent_t done) {
    Ctx *c = s->ctx;
    sw::MixGroup *hg;
    sw_status st = SW_OK;
    DescRing &ring = s->ring;
    const int slot = ring.next;
    ring.next = (ring.next + 1) % DescRing::kSlots;
    if (ring.used[slot]) {
        hipError_t e = hipEventSynchronize(ring.ev[slot]);
        if (e != hipSuccess) return e;
    }
    ring.used[slot] = true;
    hg = ring.host + 2 * slot;
    sw::MixGroup &gr = hg[0], &gi = hg[1];
    gr.nitems = 0;
    gi.nitems = (int)rs.size();
    int64_t first = 0;
    const sw::Geo g = rs[0]->geo;
    const sw::AngleTable *t;
    st = get_table(c, g.n, &t);
    if (st != SW_OK) return hipErrorUnknown;
    const sw::ProjPlan *pp;
    st = get_plan(c, g.L, g.n, &pp);
    if (st != SW_OK) return hipErrorUnknown;
    std::vector<uint64_t> keys_done;
    // a step holds one geometry: all items take the same alignment kernel
    const bool fast = sw::align128_supported(g) && !c->generic_align;
    for (size_t i = 0; i < rs.size(); ++i) {
        Req *q = rs[i];
        sw::MixItem a{};
        a.L = g.L;
        a.n = g.n;
        a.Q = g.Q;
        a.levels = g.levels;
        auto tr = c->tile_R.find(g.L);
        a.R = tr != c->tile_R.end() ? tr->second : 0;
        a.d32 = t->d32;
        a.d64 = t->d64;
        a.perm = pp->perm;
        a.trow = pp->trow;
        a.mode = s->cfg.mode;
        a.bf16 = s->cfg.prec == SW_PREC_BF16_SPLIT;
        a.top_k = s->cfg.top_k;
        a.ref_qt = (const float *)(s->base + q->o_rqt);
        a.ref_aux = (const double *)(s->base + q->o_raux);
        a.ref_spec = (float2 *)(s->base + q->o_spec);
        a.gam = fast ? (float2 *)(s->base + q->o_gam) : nullptr;
        a.img = (const float *)(s->base + q->o_img);
        a.qt = (float *)(s->base + q->o_qt);
        a.aux = (double *)(s->base + q->o_aux);
        a.out = (sw::Result *)(s->base + q->o_out);
        a.first = first;
        a.count = q->r.N;
        first += q->r.N;
        gi.items[i] = a;
        const bool dup = q->ref_key &&
                         std::find(keys_done.begin(), keys_done.end(), q->ref_key) != keys_done.end();
        if (q->ref_compute && !dup) {
            sw::MixItem r = a;
            r.img = (const float *)(s->base + q->o_ref);
            r.qt = (float *)(s->base + q->o_rqt);
            r.aux = (double *)(s->base + q->o_raux);
            r.first = gr.nitems;
            r.count = 1;
            r.gam = nullptr;
            r.spec = 1;  // writes this request's reference spectrum
            gi.items[i].spec = 1;
            gr.items[gr.nitems++] = r;
            if (q->ref_key) keys_done.push_back(q->ref_key);
        }
    }
    gr.total = gr.nitems;
    gi.total = first;
    gr.split = 0;
    gi.split = fast ? first : 0;
    sw::MixLaunch m = sw::plan_mixed(gi.items, gi.nitems, c->knobs_for({{g.L, first}}));
    for (int i = 0; i < gr.nitems; ++i) {
        gr.items[i].R = gi.items[0].R;
        gr.items[i].TC = gi.items[0].TC;
        gr.items[i].fused = gi.items[0].fused;
    }
    if (gr.nitems == 0) gr.items[0] = gi.items[0];  // keeps the binary search in range
    hipError_t e = hipSuccess;
    if (m.slot_floats > s->slot_floats) {
        e = hipStreamSynchronize(s->comp_s);
        if (e != hipSuccess) return e;
        if (s->d_slots) (void)hipFree(s->d_slots);
        s->d_slots = nullptr;
        e = hipMalloc(&s->d_slots, sizeof(float) * (size_t)m.slot_floats * s->grid);
        if (e != hipSuccess) return e;
        s->slot_floats = m.slot_floats;
        for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
        s->graphs.clear();
    }
    for (Req *q : rs)
        if (q->copied && (e = hipStreamWaitEvent(s->comp_s, q->copied, 0)) != hipSuccess) return e;
    e = hipMemcpyAsync(s->d_groups, hg, 2 * sizeof(sw::MixGroup), hipMemcpyHostToDevice, s->comp_s);
    if (e == hipSuccess) e = hipEventRecord(ring.ev[slot], s->comp_s);
    if (e != hipSuccess) return e;
    sw::MixLaunch mm = m;
    mm.slot_floats = s->slot_floats;
    if (s->cfg.use_graphs) {
        const std::vector<int> key{g.L, g.n, g.Q, g.levels, gi.items[0].R, gi.items[0].TC,
                                   gi.items[0].fused, (int)mm.tables_lds, (int)mm.align_lds,
                                   mm.region_floats, mm.lmax, mm.nmax, mm.tpw, mm.align_bpc};
        auto it = s->graphs.find(key);
        if (it == s->graphs.end()) {
            sw::prepare_mixed();
            hipGraph_t graph;
            e = hipStreamBeginCapture(s->comp_s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            hipError_t le = sw::launch_mixed(s->d_groups, s->d_groups + 1, mm, s->d_cnt, s->d_slots,
                                             s->grid, s->comp_s);
            e = hipStreamEndCapture(s->comp_s, &graph);
            if (le != hipSuccess) return le;
            if (e != hipSuccess) return e;
            hipGraphExec_t exec;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return e;
            it = s->graphs.emplace(key, exec).first;
        }
        e = hipGraphLaunch(it->second, s->comp_s);
        ++s->st.graph_launches;
    } else {
        e = sw::launch_mixed(s->d_groups, s->d_groups + 1, mm, s->d_cnt, s->d_slots, s->grid,
                             s->comp_s);
    }
    if (e != hipSuccess) return e;
    for (Req *q : rs) {
        e = hipMemcpyAsync(q->host_out, s->base + q->o_out, sizeof(sw_result) * (size_t)q->r.N,
                           hipMemcpyDeviceToHost, s->comp_s);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(done, s->comp_s);
}

void scheduler(Server *s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stopping) {
            // drop what has not reached the device; finish what has
            for (uint64_t tk : s->pending) s->reqs.erase(tk);
            s->pending.clear();
            for (uint64_t tk : s->admitted) {
                release_request(s, s->reqs[tk].get());
                s->reqs.erase(tk);
            }
            s->admitted.clear();
        }
        // 1. completions
        while (!s->steps.empty()) {
            Step &stp = s->steps.front();
            const hipError_t q = hipEventQuery(stp.done);
            if (q == hipErrorNotReady) break;
            for (uint64_t tk : stp.tickets) {
                auto it = s->reqs.find(tk);
                if (it == s->reqs.end()) continue;
                Req *r = it->second.get();
                const bool ref_ok = q == hipSuccess && reference_ok(s, r);
                if (q != hipSuccess) producer_failed(s, r);
                release_request(s, r);
                if (q != hipSuccess || !ref_ok) {
                    r->state = RState::Failed;
                    r->err = q != hipSuccess ? hipGetErrorString(q)
                                             : "the step computing its cached reference failed";
                    ++s->st.failed;
                } else if (r->cancel) {
                    r->state = RState::Cancelled;
                    ++s->st.cancelled;
                    s->pins.put(r->host_out, r->host_cap);
                    r->host_out = nullptr;
                    s->reqs.erase(it);
                } else {
                    r->state = RState::Done;
                    ++s->st.completed;
                }
            }
            (void)hipEventDestroy(stp.done);
            s->steps.pop_front();
            s->cv.notify_all();
        }
        if (s->stopping && s->steps.empty()) break;
        // 2. admission
        std::vector<Req *> fresh;
        if (!s->stopping) admit(s, fresh);
        // 3. copies of the newly admitted requests (outside the lock)
        if (!fresh.empty()) {
            lk.unlock();
            for (Req *q : fresh) {
                if (!q->host_out) continue;  // finished as a failure at launch
                const size_t L2 = (size_t)q->geo.L * q->geo.L;
                hipError_t e = hipMemcpyAsync(s->base + q->o_img, q->r.imgs,
                                              4 * (size_t)q->r.N * L2, hipMemcpyHostToDevice,
                                              s->copy_s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(s->base + q->o_ref, q->r.ref_img, 4 * L2,
                                       hipMemcpyHostToDevice, s->copy_s);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&q->copied, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(q->copied, s->copy_s);
                if (e != hipSuccess) q->err = hipGetErrorString(e);
                else if (q->ticket == s->ctx->serve_fail_ticket)
                    q->err = "injected copy failure (serve_fail_ticket)";
            }
            lk.lock();
        }
        // 4. steps: admitted requests grouped by geometry, oldest first
        while (!s->admitted.empty()) {
            std::vector<Req *> batch;
            std::vector<uint64_t> rest;
            const sw::Geo g0 = s->reqs[s->admitted.front()]->geo;
            for (uint64_t tk : s->admitted) {
                Req *q = s->reqs[tk].get();
                const bool same = q->geo.L == g0.L && q->geo.n == g0.n && q->geo.Q == g0.Q &&
                                  q->geo.levels == g0.levels;
                if (same && (int)batch.size() < s->cfg.max_per_step && q->err.empty())
                    batch.push_back(q);
                else rest.push_back(tk);
            }
            // requests whose copy failed are finished as failures
            for (auto it = rest.begin(); it != rest.end();) {
                Req *q = s->reqs[*it].get();
                if (!q->err.empty()) {
                    producer_failed(s, q);
                    release_request(s, q);
                    q->state = RState::Failed;
                    ++s->st.failed;
                    it = rest.erase(it);
                } else {
                    ++it;
                }
            }
            s->admitted = rest;
            if (batch.empty()) break;
            assign_producers(s, batch);
            Step stp;
            hipError_t e = hipEventCreateWithFlags(&stp.done, hipEventDisableTiming);
            lk.unlock();
            if (e == hipSuccess) e = issue_step(s, batch, stp.done);
            lk.lock();
            for (Req *q : batch) {
                stp.tickets.push_back(q->ticket);
                q->state = RState::Launched;
            }
            if (e != hipSuccess) {
                for (Req *q : batch) {
                    producer_failed(s, q);
                    release_request(s, q);
                    q->state = RState::Failed;
                    q->err = hipGetErrorString(e);
                    ++s->st.failed;
                }
                if (stp.done) (void)hipEventDestroy(stp.done);
                s->cv.notify_all();
                continue;
            }
            ++s->st.steps;
            s->steps.push_back(std::move(stp));
        }
        // 5. wait: briefly while work is in flight, else until woken
        if (!s->steps.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        } else if (!s->stopping) {
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

void stop_server(Ctx *c) {
    Server *s = c ? c->server : nullptr;
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    DeviceGuard dg(c->device);
    if (s->comp_s) (void)hipStreamSynchronize(s->comp_s);
    if (s->copy_s) (void)hipStreamSynchronize(s->copy_s);
    for (auto &kv : s->reqs) {
        release_request(s, kv.second.get());
        s->pins.put(kv.second->host_out, kv.second->host_cap);
        kv.second->host_out = nullptr;
    }
    s->pins.clear();
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (int i = 0; i < DescRing::kSlots; ++i)
        if (s->ring.ev[i]) (void)hipEventDestroy(s->ring.ev[i]);
    if (s->ring.host) (void)hipHostFree(s->ring.host);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->d_groups) (void)hipFree(s->d_groups);
    if (s->d_cnt) (void)hipFree(s->d_cnt);
    if (s->base) (void)hipFree(s->base);
    if (s->comp_s) (void)hipStreamDestroy(s->comp_s);
    if (s->copy_s) (void)hipStreamDestroy(s->copy_s);
    delete s;
    c->server = nullptr;
}

}  // namespace swh

using namespace swh;

extern "C" {

sw_status sw_serve_start(void *ctx, const sw_serve_cfg *cfg) {
    if (!ctx || !cfg) return fail(SW_E_INVALID, "ctx or cfg is NULL");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (c->server) return fail(SW_E_INVALID, "serving already started on this context");
    if (cfg->hbm_budget_bytes < ((size_t)1 << 20))
        return fail(SW_E_INVALID, "hbm_budget_bytes below 1 MiB");
    if (cfg->prec != SW_PREC_FP32 && cfg->prec != SW_PREC_BF16_SPLIT)
        return fail(SW_E_INVALID, "prec = %d is not a sw_precision value", cfg->prec);
    if (cfg->mode != SW_MODE_ROT_TRANS && cfg->mode != SW_MODE_ROT_ONLY)
        return fail(SW_E_INVALID, "mode = %d is not a sw_mode value", cfg->mode);
    auto *s = new (std::nothrow) Server;
    if (!s) return fail(SW_E_NOMEM, "out of host memory");
    s->cfg = *cfg;
    if (s->cfg.max_slots <= 0 || s->cfg.max_slots > sw::kMaxMix * 4) s->cfg.max_slots = sw::kMaxMix;
    if (s->cfg.max_per_step <= 0 || s->cfg.max_per_step > s->cfg.max_slots)
        s->cfg.max_per_step = s->cfg.max_slots;
    if (s->cfg.max_per_step > sw::kMaxMix) s->cfg.max_per_step = sw::kMaxMix;
    if (s->cfg.max_queue <= 0) s->cfg.max_queue = 4096;
    if (s->cfg.top_k == 0) s->cfg.top_k = s->cfg.prec == SW_PREC_BF16_SPLIT ? 4 : 1;
    if (s->cfg.top_k < 1 || s->cfg.top_k > sw::kMaxTopK) {
        delete s;
        return fail(SW_E_INVALID, "top_k = %d outside [1, %d]", cfg->top_k, sw::kMaxTopK);
    }
    s->ctx = c;
    s->grid = 2 * c->cu_count;
    DeviceGuard dg(c->device);
    hipError_t e = hipMalloc((void **)&s->base, cfg->hbm_budget_bytes);
    if (e != hipSuccess) {
        delete s;
        return fail(SW_E_NOMEM, "hipMalloc(%zu) for the serving arena failed", cfg->hbm_budget_bytes);
    }
    s->arena.init(cfg->hbm_budget_bytes);
    s->st.arena_size = cfg->hbm_budget_bytes;
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_groups, 2 * sizeof(sw::MixGroup));
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_cnt, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->comp_s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->ring.host, sizeof(sw::MixGroup) * 2 * DescRing::kSlots);
    for (int i = 0; i < DescRing::kSlots && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&s->ring.ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        c->server = s;
        stop_server(c);
        return hip_fail(e, "serving set-up");
    }
    c->server = s;
    s->th = std::thread(scheduler, s);
    return SW_OK;
}

sw_status sw_serve_submit(void *ctx, const sw_request *r, uint64_t *ticket) {
    Server *s;
    sw_status st = require_server(static_cast<Ctx *>(ctx), &s);
    if (st != SW_OK) return st;
    if (!r || !ticket) return fail(SW_E_INVALID, "request or ticket pointer is NULL");
    sw::Geo g;
    if ((st = check_geom(&r->geom, &g)) != SW_OK) return st;
    if (r->N < 1) return fail(SW_E_INVALID, "a request needs at least one image");
    if (!r->ref_img || !r->imgs) return fail(SW_E_INVALID, "ref_img or imgs is NULL");
    if (s->cfg.top_k > g.n) return fail(SW_E_INVALID, "top_k exceeds n_angles");
    const size_t need = request_bytes(*r, g, true) + up(4 * (size_t)g.Q * g.n) + up(32);
    if (need > s->cfg.hbm_budget_bytes)
        return fail(SW_E_NOMEM, "request needs %zu bytes, budget is %zu", need,
                    s->cfg.hbm_budget_bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(SW_E_INVALID, "serving is stopping");
    if ((int64_t)s->pending.size() >= s->cfg.max_queue)
        return fail(SW_E_BUSY, "%zu requests already waiting", s->pending.size());
    auto q = std::make_unique<Req>();
    q->ticket = s->next_ticket++;
    q->r = *r;
    q->geo = g;
    *ticket = q->ticket;
    s->pending.push_back(q->ticket);
    s->reqs[q->ticket] = std::move(q);
    ++s->st.submitted;
    s->cv.notify_all();
    return SW_OK;
}

sw_status sw_serve_poll(void *ctx, uint64_t ticket, sw_result *out) {
    Server *s;
    sw_status st = require_server(static_cast<Ctx *>(ctx), &s);
    if (st != SW_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(SW_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Req *q = it->second.get();
    if (q->state == RState::Failed) {
        std::string msg = q->err;
        s->pins.put(q->host_out, q->host_cap);
        s->reqs.erase(it);
        return fail(SW_E_DEVICE, "request failed: %s", msg.c_str());
    }
    if (q->state != RState::Done) return SW_NOT_READY;
    if (out) std::memcpy(out, q->host_out, sizeof(sw_result) * (size_t)q->r.N);
    s->pins.put(q->host_out, q->host_cap);
    s->reqs.erase(it);
    return SW_OK;
}

sw_status sw_serve_cancel(void *ctx, uint64_t ticket) {
    Server *s;
    sw_status st = require_server(static_cast<Ctx *>(ctx), &s);
    if (st != SW_OK) return st;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(SW_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Req *q = it->second.get();
    if (q->state == RState::Pending) {
        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), ticket));
        s->reqs.erase(it);
        ++s->st.cancelled;
        return SW_OK;
    }
    if (q->state == RState::Done || q->state == RState::Failed) {
        s->pins.put(q->host_out, q->host_cap);
        s->reqs.erase(it);
        ++s->st.cancelled;
        return SW_OK;
    }
    // admitted or on the device: wait for its step, after which the host
    // arrays are no longer read and the results are dropped
    q->cancel = true;
    s->cv.wait(lk, [&] {
        auto f = s->reqs.find(ticket);
        return f == s->reqs.end() || f->second->state == RState::Failed || s->stopping;
    });
    auto f = s->reqs.find(ticket);
    if (f != s->reqs.end()) {
        s->pins.put(f->second->host_out, f->second->host_cap);
        s->reqs.erase(f);
    }
    return SW_OK;
}

sw_status sw_serve_stats_get(void *ctx, sw_serve_stats *out) {
    Server *s;
    sw_status st = require_server(static_cast<Ctx *>(ctx), &s);
    if (st != SW_OK) return st;
    if (!out) return fail(SW_E_INVALID, "stats pointer is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->pending = (int64_t)s->pending.size();
    int64_t inflight = (int64_t)s->admitted.size();
    for (auto &stp : s->steps) inflight += (int64_t)stp.tickets.size();
    out->in_flight = inflight;
    out->arena_used = s->arena.used();
    out->arena_peak = s->arena.peak();
    return SW_OK;
}

sw_status sw_serve_stop(void *ctx) {
    if (!ctx) return fail(SW_E_INVALID, "ctx is NULL");
    stop_server(static_cast<Ctx *>(ctx));
    return SW_OK;
}

}  // extern "C"
