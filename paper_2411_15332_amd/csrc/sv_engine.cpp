// Serving engine: continuous batching of independent circuit evaluations
// (contract in include/sv.h). Host-side scheduler in C++; every state update
// and readout runs in the gfx950 kernels.
//
// Small states share one launch with one workgroup per request (the state
// never leaves LDS). Larger states are grouped by identical circuit and run as
// batched fused passes. Groups go to a pool of HIP streams (default priority);
// a finished group's stream immediately takes the oldest queued requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <cstring>
#include <deque>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sv.h"
#include "sv_internal.hpp"
#include "sv_kernels.hpp"
#include "sv_planner.hpp"

using namespace sv;

namespace {

struct Template {
    int n = 0, qubit = 0;
    Lowering low;            // composite kinds lowered
    std::vector<sv_gate> gates;
    size_t n_params = 0;     // caller's parameters plus derived columns
    bool small = false;
    Plan plan;
    // stepped engine: the plan's passes and layouts in the plan arena
    bool in_arena = false;
    uint64_t passes_off = 0, layouts_off = 0;
};

struct Request {
    uint64_t id = 0;
    std::shared_ptr<Template> t;
    std::vector<double> params;
};

// Remove the entries at the ascending, distinct indices `idx` from `q`,
// keeping the order of the rest, in one pass: a prefix is erased from the
// front; otherwise the rest moves down once. (One erase per entry would move
// the queue once per entry: quadratic in the group size.)
template <typename Q>
void erase_indices(Q &q, const std::vector<size_t> &idx) {
    if (idx.empty()) return;
    if (idx.back() + 1 == idx.size()) {
        q.erase(q.begin(), q.begin() + (long)idx.size());
        return;
    }
    size_t w = idx[0], k = 0;
    for (size_t i = idx[0]; i < q.size(); ++i) {
        if (k < idx.size() && idx[k] == i) {
            ++k;
            continue;
        }
        q[w++] = std::move(q[i]);
    }
    q.erase(q.begin() + (long)w, q.end());
}

// A few host threads that share one batch of independent jobs with the
// calling thread (the op records of a step's newly admitted requests).
class JobPool {
public:
    explicit JobPool(int workers) {
        for (int i = 0; i < workers; ++i) th_.emplace_back([this] { loop(); });
    }
    ~JobPool() {
        {
            std::lock_guard<std::mutex> l(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // Runs job(i) for i in [0, n) on the workers and the caller; returns when all are done.
    void run(size_t n, const std::function<void(size_t)> &job) {
        if (n == 0) return;
        {
            std::lock_guard<std::mutex> l(mu_);
            job_ = &job;
            n_ = n;
            next_.store(0);
            left_ = n;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> l(mu_);
        done_cv_.wait(l, [this] { return left_ == 0; });
        job_ = nullptr;
    }

private:
    void work() {
        for (;;) {
            const size_t i = next_.fetch_add(1);
            if (i >= n_) return;
            (*job_)(i);
            std::lock_guard<std::mutex> l(mu_);
            if (--left_ == 0) done_cv_.notify_all();
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return stop_ || (gen_ != seen && job_ != nullptr); });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(size_t)> *job_ = nullptr;
    size_t n_ = 0, left_ = 0;
    std::atomic<size_t> next_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// Stepped engine: a request on the GPU. It runs pass `next` of its plan in
// the next step; its op records sit in the plan arena's ring at ops_off.
struct Active {
    uint64_t id = 0;
    std::shared_ptr<Template> t;
    void *state = nullptr;
    size_t bytes = 0;
    uint64_t ops_off = 0;
    size_t ring_entry = 0;   // its allocation in the ring (sequence number)
    uint64_t ring_bytes = 0;
    int next = 0;
};

// Ring allocator over [rb, re) of the plan arena: allocations are placed in
// order and released in any order; space is reused once every older
// allocation is released too (requests finish roughly in arrival order).
struct Ring {
    uint64_t rb = 0, re = 0, head = 0, tail = 0;
    struct Ent { uint64_t off, size; bool freed; };
    std::deque<Ent> live;
    uint64_t first_seq = 0;  // sequence number of live.front()
    bool alloc(uint64_t size, uint64_t &off, uint64_t &seq) {
        size = (size + 255) & ~(uint64_t)255;
        if (live.empty()) head = tail = rb;
        if (head >= tail) {
            if (head + size <= re) off = head;
            else if (rb + size <= tail || (live.empty() && rb + size <= re)) off = rb;
            else return false;
        } else {
            if (head + size <= tail) off = head;
            else return false;
        }
        head = off + size;
        seq = first_seq + live.size();
        live.push_back({off, size, false});
        return true;
    }
    void release(uint64_t seq) {
        live[(size_t)(seq - first_seq)].freed = true;
        while (!live.empty() && live.front().freed) {
            live.pop_front();
            ++first_seq;
        }
        tail = live.empty() ? head : live.front().off;
    }
};

// One step in flight: its device scratch (partial sums, results), the
// requests it completes and where their results land. Its tables sit in the
// plan arena's ring (released with the step).
struct StepSlot {
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t ops_bytes = 0;             // op record bytes of the requests it completes
    char *d_buf = nullptr;
    size_t d_cap = 0;
    double *h_res = nullptr;
    size_t h_res_cap = 0;
    std::vector<uint64_t> ids;          // results in h_res order
    std::vector<uint64_t> ring_seqs;    // op records to release when done
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> ids;
    sv_state_s h;                     // runs the larger-state plans on this stream
    void *d_state = nullptr;
    size_t d_state_cap = 0;
    void *h_stage = nullptr;          // small-state group upload
    size_t h_stage_cap = 0;
    void *d_stage = nullptr;
    size_t d_stage_cap = 0;
    double *d_res = nullptr;
    size_t d_res_cap = 0;
    double *h_res = nullptr;
    size_t h_res_cap = 0;
};

}  // namespace

struct sv_engine_s {
    sv_dtype dt = SV_C64;
    int max_batch = 64;
    int n_streams = 4;
    size_t budget = 0;
    size_t amp_bytes = 8;
    int small_max = kSmallMaxQubitsC64;
    int device = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::deque<Request> queue;        // stepped mode: the larger states only
    std::deque<Request> small_queue;  // stepped mode: the small states
    std::unordered_map<std::string, std::shared_ptr<Template>> templates;
    std::vector<std::shared_ptr<Template>> registered;   // sv_engine_register handles
    std::deque<std::pair<uint64_t, double>> finished;
    size_t bytes_held = 0;
    int64_t completed = 0, groups = 0, largest = 0, deferred = 0, small_groups = 0;
    // stepped mode (SV_ENGINE_STEPPED): larger states advance one pass per step
    bool stepped = false;
    hipStream_t step_stream = nullptr;
    hipMemPool_t pool = nullptr;   // state memory; keeps what is freed for the next requests
    // finished requests' state buffers by n, reused by the next requests of
    // that size in stream order (a pool allocation and free per request cost
    // tens of microseconds of host time); counted against the budget
    std::vector<void *> free_states[64];
    size_t bytes_cached = 0;
    char *d_arena = nullptr;
    char *h_arena = nullptr;     // pinned mirror: records are written here, then copied
    uint64_t arena_cap = 0, tmpl_used = 0, tmpl_cap = 0;
    Ring ring;
    std::deque<Active> active;   // admission order
    std::vector<StepSlot> steps;
    size_t next_step = 0;        // ring of step slots
    std::deque<size_t> step_order;   // busy step slots, oldest first
    int max_active = 64;
    std::vector<std::pair<uint64_t, uint64_t>> uploads;   // arena ranges to copy with the next step
    uint64_t ops_live = 0;   // ring bytes held by active requests' op records (at most half the ring,
                             // so that step tables always find room)
    std::unique_ptr<JobPool> jobs;   // builds admitted requests' op records and small groups' constants in parallel
};

namespace {

std::string template_key(int n, int qubit, size_t n_params, const sv_gate *g, size_t ng) {
    std::string k;
    k.reserve(16 + ng * sizeof(sv_gate));
    const int32_t hdr[3] = {n, qubit, (int32_t)n_params};
    k.append(reinterpret_cast<const char *>(hdr), sizeof hdr);
    for (size_t i = 0; i < ng; ++i) {
        sv_gate c = g[i];
        if (c.param >= 0) c.angle = 0.0;   // referenced angles come from the parameters
        k.append(reinterpret_cast<const char *>(&c), sizeof c);
    }
    return k;
}

PlanOptions engine_plan_options(const sv_engine_s *e, bool small) {
    sv_state_s tmp;
    tmp.dt = e->dt;
    PlanOptions o = plan_options(&tmp);
    o.basis_known = true;   // every request starts from |0...0>, generated by
    o.basis_j = 0;          // the first pass of a tiled plan
    o.gen_basis = true;
    o.small_mode = small ? 2 : 1;
    return o;
}

// Make room for `need` state bytes on slot `s`: release idle slots' buffers if
// the budget requires it. Returns false when the groups in flight hold too much.
bool reserve_state(sv_engine_s *e, Slot &s, size_t need) {
    if (s.d_state_cap >= need) return true;
    auto over = [&](size_t extra) { return e->budget && e->bytes_held - s.d_state_cap + extra > e->budget; };
    if (over(need)) {
        for (auto &o : e->slots) {
            if (o.get() == &s || o->busy || !o->d_state) continue;
            hipFreeAsync(o->d_state, o->stream);
            e->bytes_held -= o->d_state_cap;
            o->d_state = nullptr;
            o->d_state_cap = 0;
            if (!over(need)) break;
        }
        if (over(need)) return false;
    }
    if (s.d_state) {
        hipFreeAsync(s.d_state, s.stream);
        e->bytes_held -= s.d_state_cap;
        s.d_state = nullptr;
        s.d_state_cap = 0;
    }
    if (hipMallocAsync(&s.d_state, need, s.stream) != hipSuccess) {
        s.d_state = nullptr;
        return false;
    }
    s.d_state_cap = need;
    e->bytes_held += need;
    return true;
}

sv_status ensure_pinned(void **p, size_t *cap, size_t need) {
    return ensure_host_buf(p, cap, need, "hipHostMalloc(engine)");
}

sv_status launch_small_group(sv_engine_s *e, Slot &s, std::vector<Request> &grp) {
    const bool f32 = e->dt == SV_C64;
    const size_t rb = f32 ? 4 : 8;
    // ops once per distinct circuit; constants once per request
    std::unordered_map<const Template *, int> op_at;
    std::vector<SmallOp> ops;
    std::vector<SmallJob> jobs(grp.size());
    uint64_t creals = 0;
    for (size_t i = 0; i < grp.size(); ++i) {
        const Template *t = grp[i].t.get();
        auto it = op_at.find(t);
        if (it == op_at.end()) {
            it = op_at.emplace(t, (int)ops.size()).first;
            ops.insert(ops.end(), t->plan.sops.begin(), t->plan.sops.end());
        }
        jobs[i].n = t->n;
        jobs[i].qubit = t->qubit;
        jobs[i].op_begin = it->second;
        jobs[i].n_ops = (int)t->plan.sops.size();
        jobs[i].const_begin = creals;
        jobs[i].pad = 0;
        creals += t->plan.cstride;
    }
    const size_t o_jobs = 0;
    const size_t o_ops = align_up(jobs.size() * sizeof(SmallJob), 256);
    const size_t o_c = align_up(o_ops + std::max<size_t>(1, ops.size()) * sizeof(SmallOp), 256);
    const size_t total = align_up(o_c + std::max<uint64_t>(1, creals) * rb, 256);
    sv_status st = ensure_pinned(&s.h_stage, &s.h_stage_cap, total);
    if (st != SV_OK) return st;
    st = ensure_device_buf(&s.d_stage, &s.d_stage_cap, total, "hipMalloc(engine stage)");
    if (st != SV_OK) return st;
    char *h = static_cast<char *>(s.h_stage);
    std::memcpy(h + o_jobs, jobs.data(), jobs.size() * sizeof(SmallJob));
    if (!ops.empty()) std::memcpy(h + o_ops, ops.data(), ops.size() * sizeof(SmallOp));
    // each request's constants into its own range of the staging buffer; on
    // the host thread pool where the engine has one (stepped mode)
    auto consts_of = [&](size_t i) {
        const Template &t = *grp[i].t;
        if (t.plan.cstride == 0) return;
        materialize_consts(t.plan, t.gates.data(), grp[i].params.data(), t.n_params, 1, f32,
                           h + o_c + jobs[i].const_begin * rb);
    };
    if (e->jobs) {
        std::atomic<bool> bad{false};
        e->jobs->run(grp.size(), [&](size_t i) {
            try {
                consts_of(i);
            } catch (...) {   // no exception may leave a worker thread
                bad.store(true);
            }
        });
        if (bad.load()) return fail(SV_EUNSUPPORTED, "serving engine: constants could not be built");
    } else {
        for (size_t i = 0; i < grp.size(); ++i) consts_of(i);
    }
    SV_HIP(hipMemcpyAsync(s.d_stage, s.h_stage, total, hipMemcpyHostToDevice, s.stream), "hipMemcpyAsync(jobs)");
    st = ensure_device_buf(reinterpret_cast<void **>(&s.d_res), &s.d_res_cap, grp.size() * sizeof(double),
                           "hipMalloc(results)");
    if (st != SV_OK) return st;
    char *d = static_cast<char *>(s.d_stage);
    SV_HIP(launch_small_jobs((int)e->dt, reinterpret_cast<const SmallJob *>(d + o_jobs), (int)grp.size(),
                             reinterpret_cast<const SmallOp *>(d + o_ops), d + o_c, s.d_res, s.stream),
           "launch small jobs");
    ++e->small_groups;
    return SV_OK;
}

sv_status launch_large_group(sv_engine_s *e, Slot &s, std::vector<Request> &grp) {
    const Template &t = *grp[0].t;
    const int k = (int)grp.size();
    const uint64_t N = 1ull << t.n;
    s.h.n = t.n;
    s.h.dt = e->dt;
    s.h.batch = k;
    s.h.amp_bytes = e->amp_bytes;
    s.h.buf = s.d_state;
    s.h.owned = false;
    s.h.stream = s.stream;
    s.h.device = e->device;
    std::vector<double> params((size_t)k * std::max<size_t>(1, t.n_params), 0.0);
    for (int i = 0; i < k; ++i)
        std::copy(grp[i].params.begin(), grp[i].params.end(), params.begin() + (size_t)i * t.n_params);
    if (t.plan.small || t.plan.passes.empty() || !(t.plan.passes[0].flags & PASS_GENERATES))
        SV_HIP(launch_fill_basis((int)e->dt, s.d_state, N, k, 0, s.stream), "launch fill");
    sv_status st = run_plan(&s.h, s.d_state, k, t.plan, t.gates.data(), params.data(), t.n_params);
    if (st != SV_OK) return st;
    const size_t np = reduce_partials_size(t.n) * (size_t)k;
    st = ensure_device_buf(reinterpret_cast<void **>(&s.h.d_red), &s.h.d_red_cap, np * sizeof(double),
                           "hipMalloc(reduce)");
    if (st != SV_OK) return st;
    st = ensure_device_buf(reinterpret_cast<void **>(&s.d_res), &s.d_res_cap, (size_t)k * sizeof(double),
                           "hipMalloc(results)");
    if (st != SV_OK) return st;
    SV_HIP(launch_reduce((int)e->dt, s.d_state, t.n, k, t.qubit, s.h.d_red, s.d_res, s.stream),
           "launch reduce");
    return SV_OK;
}

sv_status retire(sv_engine_s *e) {
    for (auto &sp : e->slots) {
        Slot &s = *sp;
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return hip_fail(q, "engine group");
        for (size_t i = 0; i < s.ids.size(); ++i) e->finished.emplace_back(s.ids[i], s.h_res[i]);
        e->completed += (int64_t)s.ids.size();
        s.ids.clear();
        s.busy = false;
    }
    return SV_OK;
}

sv_status launch_ready(sv_engine_s *e) {
    // stepped mode: these slots serve the small states, from their own queue
    std::deque<Request> &queue = e->stepped ? e->small_queue : e->queue;
    for (auto &sp : e->slots) {
        Slot &s = *sp;
        if (s.busy) continue;
        if (queue.empty()) break;
        const size_t fi = 0;
        const Request &front = queue[fi];
        bool small = front.t->small;
        std::vector<size_t> pick;
        for (size_t i = fi; i < queue.size() && (int)pick.size() < e->max_batch; ++i) {
            const Request &r = queue[i];
            if (small ? r.t->small : r.t == front.t) pick.push_back(i);
        }
        if (!small) {
            const size_t per = ((size_t)1 << front.t->n) * e->amp_bytes;
            size_t k = pick.size();
            if (e->budget) {
                // admission by HBM footprint: shrink the group to what fits
                size_t others = e->bytes_held - s.d_state_cap;
                for (auto &o : e->slots)
                    if (o.get() != &s && !o->busy) others -= o->d_state_cap;  // idle buffers can be released
                const size_t room = e->budget > others ? e->budget - others : 0;
                k = std::min(k, room / per);
            }
            if (k == 0 || !reserve_state(e, s, k * per)) {
                ++e->deferred;
                // the group waits for memory held by groups in flight; small
                // states hold none, so they may go ahead of it
                size_t si = fi;
                while (si < queue.size() && !queue[si].t->small) ++si;
                if (si == queue.size()) break;
                pick.clear();
                for (size_t i = si; i < queue.size() && (int)pick.size() < e->max_batch; ++i)
                    if (queue[i].t->small) pick.push_back(i);
                small = true;
            } else {
                pick.resize(k);
            }
        }
        std::vector<Request> grp;
        grp.reserve(pick.size());
        for (size_t i : pick) grp.push_back(std::move(queue[i]));
        erase_indices(queue, pick);
        sv_status st = small ? launch_small_group(e, s, grp) : launch_large_group(e, s, grp);
        if (st != SV_OK) return st;
        sv_status st2 = ensure_pinned(reinterpret_cast<void **>(&s.h_res), &s.h_res_cap,
                                      grp.size() * sizeof(double));
        if (st2 != SV_OK) return st2;
        SV_HIP(hipMemcpyAsync(s.h_res, s.d_res, grp.size() * sizeof(double), hipMemcpyDeviceToHost, s.stream),
               "hipMemcpyAsync(results)");
        SV_HIP(hipEventRecord(s.done, s.stream), "hipEventRecord");
        s.ids.clear();
        for (const Request &r : grp) s.ids.push_back(r.id);
        s.busy = true;
        ++e->groups;
        e->largest = std::max<int64_t>(e->largest, (int64_t)grp.size());
    }
    return SV_OK;
}

// ------------------------------------------------------------------------
// Stepped mode: continuous batching at pass granularity. Each step is one
// launch per kernel variant that runs the next pass of every active request,
// whatever its circuit, n or depth, plus one batched readout for the requests
// the step completes. Requests join at the next step built after their
// arrival; a step's tables are small, and the per-request op records go to
// the plan arena once, at admission.

constexpr int kStepSlots = 4;                   // steps in flight
constexpr uint64_t kArenaBytes = 256ull << 20;  // plan arena (templates + op records)
constexpr uint64_t kTemplateBytes = 32ull << 20;

sv_status stepped_init(sv_engine_s *e) {
    SV_HIP(hipStreamCreateWithFlags(&e->step_stream, hipStreamNonBlocking), "engine step stream");
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = e->device;
    SV_HIP(hipMemPoolCreate(&e->pool, &props), "hipMemPoolCreate");
    uint64_t keep = ~0ull;   // never hand freed state memory back to the driver
    SV_HIP(hipMemPoolSetAttribute(e->pool, hipMemPoolAttrReleaseThreshold, &keep), "hipMemPoolSetAttribute");
    e->arena_cap = kArenaBytes;
    e->tmpl_cap = kTemplateBytes;
    SV_HIP(hipMalloc(reinterpret_cast<void **>(&e->d_arena), e->arena_cap), "hipMalloc(plan arena)");
    SV_HIP(hipHostMalloc(reinterpret_cast<void **>(&e->h_arena), e->arena_cap, hipHostMallocDefault),
           "hipHostMalloc(plan arena)");
    e->ring.rb = e->tmpl_cap;
    e->ring.re = e->arena_cap;
    e->steps.resize(kStepSlots);
    e->jobs = std::make_unique<JobPool>(3);
    for (StepSlot &S : e->steps) SV_HIP(hipEventCreateWithFlags(&S.done, hipEventDisableTiming), "hipEventCreate");
    return SV_OK;
}

// Return the cached state buffers to the pool (stream order).
void stepped_drop_cache(sv_engine_s *e) {
    for (auto &v : e->free_states) {
        for (void *p : v) hipFreeAsync(p, e->step_stream);
        v.clear();
    }
    e->bytes_cached = 0;
}

void stepped_release(sv_engine_s *e) {
    e->jobs.reset();
    if (e->step_stream) {
        hipStreamSynchronize(e->step_stream);
        for (Active &a : e->active)
            if (a.state) hipFreeAsync(a.state, e->step_stream);
        stepped_drop_cache(e);
        hipStreamSynchronize(e->step_stream);
    }
    e->active.clear();
    for (StepSlot &S : e->steps) {
        if (S.d_buf) hipFree(S.d_buf);
        if (S.h_res) hipHostFree(S.h_res);
        if (S.done) hipEventDestroy(S.done);
    }
    e->steps.clear();
    if (e->d_arena) hipFree(e->d_arena);
    if (e->h_arena) hipHostFree(e->h_arena);
    e->d_arena = e->h_arena = nullptr;
    if (e->pool) hipMemPoolDestroy(e->pool);
    e->pool = nullptr;
    if (e->step_stream) hipStreamDestroy(e->step_stream);
    e->step_stream = nullptr;
}

// Copy the template's passes and layouts into the arena (once per template).
sv_status stepped_template(sv_engine_s *e, Template &t) {
    if (t.in_arena) return SV_OK;
    const Plan &p = t.plan;
    const uint64_t pb = p.passes.size() * sizeof(DevPass), lb = p.layouts.size() * sizeof(DevLayout);
    const uint64_t need = align_up(pb, 256) + align_up(lb, 256);
    if (e->tmpl_used + need > e->tmpl_cap) return fail(SV_ENOMEM, "serving engine: too many distinct circuits");
    t.passes_off = e->tmpl_used;
    t.layouts_off = t.passes_off + align_up(pb, 256);
    std::memcpy(e->h_arena + t.passes_off, p.passes.data(), pb);
    std::memcpy(e->h_arena + t.layouts_off, p.layouts.data(), lb);
    SV_HIP(hipMemcpyAsync(e->d_arena + t.passes_off, e->h_arena + t.passes_off, need, hipMemcpyHostToDevice,
                          e->step_stream),
           "hipMemcpyAsync(template)");
    e->tmpl_used += need;
    t.in_arena = true;
    return SV_OK;
}

// Ring bytes written on the host this step, uploaded in one copy (two when
// the ring wrapped) before the step's launches.
void stepped_note_upload(sv_engine_s *e, uint64_t off, uint64_t size) {
    auto &u = e->uploads;
    if (!u.empty() && u.back().second == off) u.back().second = off + size;
    else u.emplace_back(off, off + size);
}

sv_status stepped_flush_uploads(sv_engine_s *e) {
    for (auto &r : e->uploads)
        SV_HIP(hipMemcpyAsync(e->d_arena + r.first, e->h_arena + r.first, r.second - r.first, hipMemcpyHostToDevice,
                              e->step_stream),
               "hipMemcpyAsync(plan arena)");
    e->uploads.clear();
    return SV_OK;
}

// Admit queued larger-state requests while the active set, the HBM budget
// and the arena allow: state memory (stream-ordered) and op records.
sv_status stepped_admit(sv_engine_s *e) {
    const bool f32 = e->dt == SV_C64;
    struct Mat { const Template *t; std::vector<double> params; uint64_t off; };
    std::vector<Mat> mats;
    size_t i = 0;
    while (i < e->queue.size() && (int)e->active.size() < e->max_active) {
        Request &r = e->queue[i];
        Template &t = *r.t;
        const size_t bytes = ((size_t)1 << t.n) * e->amp_bytes;
        if (e->budget && e->bytes_held + bytes > e->budget) {
            ++e->deferred;
            break;   // admission by HBM footprint: wait for running requests to finish
        }
        if (e->free_states[t.n].empty() && e->budget && e->bytes_held + e->bytes_cached + bytes > e->budget)
            stepped_drop_cache(e);   // new memory needed: cached buffers of other sizes go first
        const uint64_t ob = (uint64_t)t.plan.ops.size() * sizeof(DevOp);
        const uint64_t held = (std::max<uint64_t>(ob, 256) + 255) & ~(uint64_t)255;
        if (e->ops_live + held > (e->ring.re - e->ring.rb) / 2) break;   // wait for arena space
        uint64_t off = 0, seq = 0;
        if (!e->ring.alloc(held, off, seq)) break;
        sv_status st = stepped_template(e, t);
        if (st != SV_OK) return st;
        Active a;
        a.id = r.id;
        a.t = r.t;
        a.bytes = bytes;
        a.ops_off = off;
        a.ring_entry = seq;
        a.ring_bytes = held;
        e->ops_live += held;
        if (!e->free_states[t.n].empty()) {
            a.state = e->free_states[t.n].back();
            e->free_states[t.n].pop_back();
            e->bytes_cached -= bytes;
        } else {
            SV_HIP(hipMallocFromPoolAsync(&a.state, bytes, e->pool, e->step_stream), "hipMallocFromPoolAsync(state)");
        }
        if (ob) mats.push_back({&t, std::move(r.params), off});
        stepped_note_upload(e, off, held);   // the allocation's extent: neighbours merge
        if (t.plan.passes.empty())   // nothing to apply: the readout sees |0...0>
            SV_HIP(launch_fill_basis((int)e->dt, a.state, 1ull << t.n, 1, 0, e->step_stream), "launch fill");
        e->bytes_held += bytes;
        e->active.push_back(std::move(a));
        e->queue.erase(e->queue.begin() + (long)i);
    }
    // op records of the admitted requests, several at a time (each job writes
    // its own ring range of the pinned mirror)
    std::atomic<bool> bad{false};
    e->jobs->run(mats.size(), [&](size_t k) {
        const Mat &m = mats[k];
        try {
            materialize_ops(m.t->plan, m.t->gates.data(), m.params.data(), m.t->n_params, 1, f32,
                            e->h_arena + m.off);
        } catch (...) {   // no exception may leave a worker thread
            bad.store(true);
        }
    });
    if (bad.load()) return fail(SV_EUNSUPPORTED, "serving engine: op records could not be built");
    return SV_OK;
}

// Build and launch one step into a free step slot.
sv_status stepped_launch(sv_engine_s *e) {
    StepSlot &S = e->steps[e->next_step];
    if (S.busy) return SV_OK;
    sv_status st = stepped_admit(e);
    if (st != SV_OK) return st;
    if (e->active.empty()) return SV_OK;

    std::vector<StepReq> reqs;
    std::vector<StepItem> items[4];   // bit 0: generating pass, bit 1: pass with a 4x4
    std::vector<RedItem> reds;
    std::vector<FinItem> fins;
    std::vector<uint64_t> ids, seqs;
    std::vector<size_t> run_idx, done_idx;
    uint64_t done_ops = 0;
    uint32_t parts = 0;
    for (size_t ai = 0; ai < e->active.size(); ++ai) {
        const Active &a = e->active[ai];
        const Template &t = *a.t;
        const int np = (int)t.plan.passes.size();
        int next = a.next;
        if (next < np) {
            const DevPass &P = t.plan.passes[(size_t)next];
            if (P.w != (e->dt == SV_C128 ? kThreadBitsC128 : kThreadBitsC64))
                return fail(SV_EUNSUPPORTED, "serving engine: tile geometry of a %d-qubit plan", t.n);
            StepReq q;
            std::memset(&q, 0, sizeof q);
            q.state = a.state;
            q.passes_off = t.passes_off;
            q.layouts_off = t.layouts_off;
            q.ops_off = a.ops_off;
            q.pass = next;
            q.n = t.n;
            const uint32_t ri = (uint32_t)reqs.size();
            reqs.push_back(q);
            const int v = ((P.flags & PASS_GENERATES) ? 1 : 0) | ((P.flags & PASS_DENSE2) ? 2 : 0);
            for (uint64_t tile = 0; tile < P.tiles; ++tile) items[v].push_back({ri, (uint32_t)tile});
            run_idx.push_back(ai);
            ++next;
        }
        if (next >= np) {   // this step completes it: batched readout
            const uint32_t nblk = (uint32_t)reduce_blocks(t.n);
            const uint64_t chunk = reduce_chunk(t.n);
            for (uint32_t b = 0; b < nblk; ++b) {
                RedItem r;
                std::memset(&r, 0, sizeof r);
                r.state = a.state;
                r.chunk = chunk;
                r.blk = b;
                r.qubit = t.qubit;
                r.part = parts + b;
                reds.push_back(r);
            }
            FinItem f;
            std::memset(&f, 0, sizeof f);
            f.first = parts;
            f.count = nblk;
            f.slot = (uint32_t)ids.size();
            fins.push_back(f);
            parts += nblk;
            ids.push_back(a.id);
            seqs.push_back(a.ring_entry);
            done_idx.push_back(ai);
            done_ops += a.ring_bytes;
        }
    }

    // step tables: in the ring, uploaded with the step's op records in one
    // copy; partial sums and results live on the device only
    size_t off = 0;
    auto sec = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_req = sec(reqs.size() * sizeof(StepReq));
    size_t o_it[4];
    for (int v = 0; v < 4; ++v) o_it[v] = sec(items[v].size() * sizeof(StepItem));
    const size_t o_red = sec(reds.size() * sizeof(RedItem));
    const size_t o_fin = sec(fins.size() * sizeof(FinItem));
    const size_t up = std::max<size_t>(off, 256);
    uint64_t toff = 0, tseq = 0;
    if (!e->ring.alloc(up, toff, tseq))
        return stepped_flush_uploads(e);   // no room for the tables yet: this step is built later
    for (size_t ai : run_idx) ++e->active[ai].next;
    S.ids = std::move(ids);
    S.ring_seqs = std::move(seqs);
    S.ops_bytes = done_ops;
    S.ring_seqs.push_back(tseq);
    const uint64_t tsize = (up + 255) & ~(uint64_t)255;
    char *ht = e->h_arena + toff;
    std::memcpy(ht + o_req, reqs.data(), reqs.size() * sizeof(StepReq));
    for (int v = 0; v < 4; ++v) std::memcpy(ht + o_it[v], items[v].data(), items[v].size() * sizeof(StepItem));
    std::memcpy(ht + o_red, reds.data(), reds.size() * sizeof(RedItem));
    std::memcpy(ht + o_fin, fins.data(), fins.size() * sizeof(FinItem));
    stepped_note_upload(e, toff, tsize);
    const size_t o_part = 0;
    const size_t o_res = align_up((size_t)parts * sizeof(double), 256);
    const size_t total = std::max<size_t>(o_res + align_up(fins.size() * sizeof(double), 256), 256);
    if (S.d_cap < total) {
        if (S.d_buf) hipFree(S.d_buf);
        S.d_buf = nullptr;
        S.d_cap = 0;
        SV_HIP(hipMalloc(reinterpret_cast<void **>(&S.d_buf), total * 2), "hipMalloc(step)");
        S.d_cap = total * 2;
    }
    hipStream_t ss = e->step_stream;
    st = stepped_flush_uploads(e);
    if (st != SV_OK) return st;
    char *dt = e->d_arena + toff;
    const StepReq *d_req = reinterpret_cast<const StepReq *>(dt + o_req);
    for (int v = 0; v < 4; ++v)
        SV_HIP(launch_pass_multi((int)e->dt, e->d_arena, d_req, reinterpret_cast<const StepItem *>(dt + o_it[v]),
                                 (uint32_t)items[v].size(), (v & 1) != 0, (v & 2) != 0, ss),
               "launch step");
    if (!fins.empty()) {
        double *d_res = reinterpret_cast<double *>(S.d_buf + o_res);
        SV_HIP(launch_reduce_multi((int)e->dt, reinterpret_cast<const RedItem *>(dt + o_red), (uint32_t)reds.size(),
                                   reinterpret_cast<double *>(S.d_buf + o_part),
                                   reinterpret_cast<const FinItem *>(dt + o_fin), (uint32_t)fins.size(), d_res, ss),
               "launch step readout");
        st = ensure_pinned(reinterpret_cast<void **>(&S.h_res), &S.h_res_cap, fins.size() * sizeof(double));
        if (st != SV_OK) return st;
        SV_HIP(hipMemcpyAsync(S.h_res, d_res, fins.size() * sizeof(double), hipMemcpyDeviceToHost, ss),
               "hipMemcpyAsync(step results)");
    }
    // finished requests leave the active set; their state memory returns to
    // the pool after the readout (stream order)
    for (size_t k : done_idx) {
        Active &a = e->active[k];
        e->free_states[a.t->n].push_back(a.state);   // reused after this step's readout (stream order)
        e->bytes_cached += a.bytes;
        e->bytes_held -= a.bytes;
    }
    erase_indices(e->active, done_idx);
    SV_HIP(hipEventRecord(S.done, ss), "hipEventRecord(step)");
    S.busy = true;
    e->step_order.push_back(e->next_step);
    e->next_step = (e->next_step + 1) % e->steps.size();
    ++e->groups;
    size_t wg = 0;
    for (int v = 0; v < 4; ++v) wg += items[v].size();
    e->largest = std::max<int64_t>(e->largest, (int64_t)reqs.size());
    (void)wg;
    return SV_OK;
}

sv_status stepped_retire(sv_engine_s *e) {
    while (!e->step_order.empty()) {
        StepSlot &S = e->steps[e->step_order.front()];
        const hipError_t q = hipEventQuery(S.done);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return hip_fail(q, "engine step");
        for (size_t i = 0; i < S.ids.size(); ++i) e->finished.emplace_back(S.ids[i], S.h_res[i]);
        e->completed += (int64_t)S.ids.size();
        for (uint64_t seq : S.ring_seqs) e->ring.release(seq);
        e->ops_live -= S.ops_bytes;
        S.ops_bytes = 0;
        S.ids.clear();
        S.ring_seqs.clear();
        S.busy = false;
        e->step_order.pop_front();
    }
    return SV_OK;
}

}  // namespace

extern "C" {

static sv_status engine_create(sv_dtype dtype, int max_batch, int n_streams, size_t hbm_budget_bytes,
                               bool stepped, int max_active, sv_engine *out) {
    return guarded([&]() -> sv_status {
        if (!out) return fail(SV_EINVAL, "out is NULL");
        *out = nullptr;
        if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "unknown dtype %d", (int)dtype);
        if (max_batch < 1 || max_batch > 65535) return fail(SV_EINVAL, "max_batch %d outside 1..65535", max_batch);
        if (n_streams < 1 || n_streams > 16) return fail(SV_EINVAL, "n_streams %d outside 1..16", n_streams);
        auto *e = new (std::nothrow) sv_engine_s();
        if (!e) return fail(SV_ENOMEM, "host allocation failed");
        e->dt = dtype;
        e->max_batch = max_batch;
        e->n_streams = n_streams;
        e->budget = hbm_budget_bytes;
        e->amp_bytes = dtype == SV_C128 ? 16 : 8;
        e->small_max = dtype == SV_C128 ? kSmallMaxQubitsC128 : kSmallMaxQubitsC64;
        hipError_t err = hipGetDevice(&e->device);
        for (int i = 0; i < n_streams && err == hipSuccess; ++i) {
            auto s = std::make_unique<Slot>();
            err = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&s->done, hipEventDisableTiming);
            e->slots.push_back(std::move(s));
        }
        if (err != hipSuccess) {
            sv_engine_free(e);
            return hip_fail(err, "engine streams");
        }
        if (stepped) {
            e->stepped = true;
            e->max_active = max_active;
            sv_status st = stepped_init(e);
            if (st != SV_OK) {
                const std::string msg = sv_last_error();
                sv_engine_free(e);
                return fail(st, "%s", msg.c_str());
            }
        }
        *out = e;
        return SV_OK;
    });
}

sv_status sv_engine_create(sv_dtype dtype, int max_batch, int n_streams, size_t hbm_budget_bytes,
                           sv_engine *out) {
    return engine_create(dtype, max_batch, n_streams, hbm_budget_bytes, false, 0, out);
}

sv_status sv_engine_create_stepped(sv_dtype dtype, int max_active, int max_small_batch, int n_small_streams,
                                   size_t hbm_budget_bytes, sv_engine *out) {
    if (max_active < 1 || max_active > 65535)
        return fail(SV_EINVAL, "max_active %d outside 1..65535", max_active);
    return engine_create(dtype, max_small_batch, n_small_streams, hbm_budget_bytes, true, max_active, out);
}

sv_status sv_engine_free(sv_engine e) {
    return guarded([&]() -> sv_status {
        if (!e) return SV_OK;
        hipSetDevice(e->device);
        stepped_release(e);
        hipError_t first = hipSuccess;
        for (auto &sp : e->slots) {
            Slot &s = *sp;
            if (s.stream) {
                hipError_t r = hipStreamSynchronize(s.stream);
                if (first == hipSuccess) first = r;
            }
            if (s.d_state) hipFree(s.d_state);
            if (s.d_stage) hipFree(s.d_stage);
            if (s.d_res) hipFree(s.d_res);
            if (s.h_stage) hipHostFree(s.h_stage);
            if (s.h_res) hipHostFree(s.h_res);
            s.h.buf = nullptr;
            s.h.owned = false;
            release_handle_buffers(&s.h);
            if (s.done) hipEventDestroy(s.done);
            if (s.stream) hipStreamDestroy(s.stream);
        }
        delete e;
        if (first != hipSuccess) return hip_fail(first, "engine shutdown");
        return SV_OK;
    });
}

}  // extern "C"

namespace {

// The engine's template of a circuit (planned once per distinct circuit).
sv_status engine_template(sv_engine_s *e, int n_qubits, const sv_gate *gates, size_t n_gates,
                          size_t n_params, bool have_params, int qubit, std::shared_ptr<Template> &out) {
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d outside 1..34", n_qubits);
    if (n_qubits > 30) return fail(SV_EUNSUPPORTED, "serving requests are limited to 30 qubits");
    if (e->budget && ((size_t)1 << n_qubits) * e->amp_bytes > e->budget)
        return fail(SV_ENOMEM, "a %d-qubit state exceeds the engine's HBM budget", n_qubits);
    if (qubit < 0 || qubit >= n_qubits) return fail(SV_EINVAL, "qubit %d out of range", qubit);
    if (n_gates && !gates) return fail(SV_EINVAL, "gates is NULL");
    std::string err;
    if (!validate_gates(n_qubits, gates, n_gates, n_params, have_params, err))
        return fail(SV_EINVAL, "%s", err.c_str());
    const std::string key = template_key(n_qubits, qubit, n_params, gates, n_gates);
    auto it = e->templates.find(key);
    if (it == e->templates.end()) {
        auto t = std::make_shared<Template>();
        t->n = n_qubits;
        t->qubit = qubit;
        lower_gates(gates, n_gates, n_params, t->low);
        t->gates = t->low.gates;
        t->n_params = n_params + t->low.src.size();
        t->small = n_qubits <= e->small_max;
        t->plan = build_plan(n_qubits, t->gates.data(), t->gates.size(), engine_plan_options(e, t->small));
        if (e->stepped && !t->small && (uint64_t)t->plan.ops.size() * sizeof(DevOp) > (e->ring.re - e->ring.rb) / 4)
            return fail(SV_ENOMEM, "serving engine: the circuit's op records exceed the plan arena");
        it = e->templates.emplace(key, std::move(t)).first;
    }
    out = it->second;
    return SV_OK;
}

void engine_enqueue(sv_engine_s *e, uint64_t id, const std::shared_ptr<Template> &t, const double *params,
                    size_t n_params) {
    Request r;
    r.id = id;
    r.t = t;
    if (t->low.src.empty()) r.params.assign(params, params + n_params);
    else lower_params(t->low, params, n_params, 1, r.params);
    if (e->stepped && t->small) e->small_queue.push_back(std::move(r));
    else e->queue.push_back(std::move(r));
}

}  // namespace

extern "C" {

sv_status sv_engine_submit(sv_engine e, uint64_t id, int n_qubits, const sv_gate *gates, size_t n_gates,
                           const double *params, size_t n_params, int qubit) {
    return guarded([&]() -> sv_status {
        if (!e) return fail(SV_EINVAL, "null engine");
        if (n_params && !params) return fail(SV_EINVAL, "params is NULL");
        std::shared_ptr<Template> t;
        sv_status st = engine_template(e, n_qubits, gates, n_gates, n_params, params != nullptr || n_params == 0,
                                       qubit, t);
        if (st != SV_OK) return st;
        engine_enqueue(e, id, t, params, n_params);
        return SV_OK;
    });
}

sv_status sv_engine_register(sv_engine e, int n_qubits, const sv_gate *gates, size_t n_gates, size_t n_params,
                             int qubit, int64_t *circuit) {
    return guarded([&]() -> sv_status {
        if (!e || !circuit) return fail(SV_EINVAL, "null argument");
        std::shared_ptr<Template> t;
        sv_status st = engine_template(e, n_qubits, gates, n_gates, n_params, true, qubit, t);
        if (st != SV_OK) return st;
        for (size_t i = 0; i < e->registered.size(); ++i)
            if (e->registered[i] == t) {
                *circuit = (int64_t)i;
                return SV_OK;
            }
        *circuit = (int64_t)e->registered.size();
        e->registered.push_back(t);
        return SV_OK;
    });
}

sv_status sv_engine_submit_registered(sv_engine e, uint64_t id, int64_t circuit, const double *params,
                                      size_t n_params) {
    return guarded([&]() -> sv_status {
        if (!e) return fail(SV_EINVAL, "null engine");
        if (circuit < 0 || (size_t)circuit >= e->registered.size())
            return fail(SV_EINVAL, "unknown circuit %lld", (long long)circuit);
        const std::shared_ptr<Template> &t = e->registered[(size_t)circuit];
        const size_t want = t->n_params - t->low.src.size();
        if (n_params != want) return fail(SV_EINVAL, "circuit %lld takes %zu parameters, got %zu",
                                          (long long)circuit, want, n_params);
        if (n_params && !params) return fail(SV_EINVAL, "params is NULL");
        engine_enqueue(e, id, t, params, n_params);
        return SV_OK;
    });
}

sv_status sv_engine_poll(sv_engine e, int64_t wait_us, uint64_t *ids, double *values, size_t cap,
                         size_t *count) {
    return guarded([&]() -> sv_status {
        if (!e || !count) return fail(SV_EINVAL, "null argument");
        *count = 0;
        if (cap && (!ids || !values)) return fail(SV_EINVAL, "ids or values is NULL");
        hipSetDevice(e->device);
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            sv_status st = retire(e);
            if (st != SV_OK) return st;
            st = launch_ready(e);
            if (st != SV_OK) return st;
            if (e->stepped) {
                st = stepped_retire(e);
                if (st != SV_OK) return st;
                for (size_t k = 0; k < e->steps.size(); ++k) {   // fill the free step slots
                    const size_t before = e->step_order.size();
                    st = stepped_launch(e);
                    if (st != SV_OK) return st;
                    if (e->step_order.size() == before) break;
                }
            }
            if (!e->finished.empty() || wait_us <= 0) break;
            bool busy = !e->step_order.empty() || !e->active.empty();
            for (auto &s : e->slots) busy = busy || s->busy;
            if (!busy && e->queue.empty() && e->small_queue.empty()) break;
            const auto el = std::chrono::duration_cast<std::chrono::microseconds>(
                std::chrono::steady_clock::now() - t0).count();
            if (el >= wait_us) break;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        size_t c = 0;
        while (c < cap && !e->finished.empty()) {
            ids[c] = e->finished.front().first;
            values[c] = e->finished.front().second;
            e->finished.pop_front();
            ++c;
        }
        *count = c;
        return SV_OK;
    });
}

sv_status sv_engine_stats(sv_engine e, int64_t out[8]) {
    return guarded([&]() -> sv_status {
        if (!e || !out) return fail(SV_EINVAL, "null argument");
        int64_t inflight = (int64_t)e->active.size();
        for (auto &s : e->slots) inflight += (int64_t)s->ids.size();
        for (size_t k : e->step_order) inflight += (int64_t)e->steps[k].ids.size();
        out[0] = (int64_t)(e->queue.size() + e->small_queue.size());
        out[1] = inflight;
        out[2] = e->completed;
        out[3] = e->groups;
        out[4] = (int64_t)e->bytes_held;
        out[5] = e->largest;
        out[6] = e->deferred;
        out[7] = e->small_groups;
        return SV_OK;
    });
}

}  // extern "C"
