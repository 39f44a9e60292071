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
#include <chrono>
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
};

struct Request {
    uint64_t id = 0;
    std::shared_ptr<Template> t;
    std::vector<double> params;
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
    std::deque<Request> queue;
    std::unordered_map<std::string, std::shared_ptr<Template>> templates;
    std::deque<std::pair<uint64_t, double>> finished;
    size_t bytes_held = 0;
    int64_t completed = 0, groups = 0, largest = 0, deferred = 0, small_groups = 0;
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
    o.basis_known = true;   // every request starts from |0...0>
    o.basis_j = 0;
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
    for (size_t i = 0; i < grp.size(); ++i) {
        const Template &t = *grp[i].t;
        if (t.plan.cstride == 0) continue;
        materialize_consts(t.plan, t.gates.data(), grp[i].params.data(), t.n_params, 1, f32,
                           h + o_c + jobs[i].const_begin * rb);
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
    for (auto &sp : e->slots) {
        Slot &s = *sp;
        if (s.busy) continue;
        if (e->queue.empty()) break;
        const Request &front = e->queue.front();
        const bool small = front.t->small;
        std::vector<size_t> pick;
        for (size_t i = 0; i < e->queue.size() && (int)pick.size() < e->max_batch; ++i) {
            const Request &r = e->queue[i];
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
                break;   // wait for memory held by groups in flight
            }
            pick.resize(k);
        }
        std::vector<Request> grp;
        grp.reserve(pick.size());
        for (size_t i : pick) grp.push_back(std::move(e->queue[i]));
        for (size_t j = pick.size(); j-- > 0;) e->queue.erase(e->queue.begin() + (long)pick[j]);
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

}  // namespace

extern "C" {

sv_status sv_engine_create(sv_dtype dtype, int max_batch, int n_streams, size_t hbm_budget_bytes,
                           sv_engine *out) {
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
        *out = e;
        return SV_OK;
    });
}

sv_status sv_engine_free(sv_engine e) {
    return guarded([&]() -> sv_status {
        if (!e) return SV_OK;
        hipSetDevice(e->device);
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

sv_status sv_engine_submit(sv_engine e, uint64_t id, int n_qubits, const sv_gate *gates, size_t n_gates,
                           const double *params, size_t n_params, int qubit) {
    return guarded([&]() -> sv_status {
        if (!e) return fail(SV_EINVAL, "null engine");
        if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d outside 1..34", n_qubits);
        if (n_qubits > 30) return fail(SV_EUNSUPPORTED, "serving requests are limited to 30 qubits");
        if (qubit < 0 || qubit >= n_qubits) return fail(SV_EINVAL, "qubit %d out of range", qubit);
        if (n_gates && !gates) return fail(SV_EINVAL, "gates is NULL");
        if (n_params && !params) return fail(SV_EINVAL, "params is NULL");
        std::string err;
        if (!validate_gates(n_qubits, gates, n_gates, n_params, params != nullptr || n_params == 0, err))
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
            it = e->templates.emplace(key, std::move(t)).first;
        }
        Request r;
        r.id = id;
        r.t = it->second;
        if (it->second->low.src.empty()) r.params.assign(params, params + n_params);
        else lower_params(it->second->low, params, n_params, 1, r.params);
        e->queue.push_back(std::move(r));
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
            if (!e->finished.empty() || wait_us <= 0) break;
            bool busy = false;
            for (auto &s : e->slots) busy = busy || s->busy;
            if (!busy && e->queue.empty()) break;
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
        int64_t inflight = 0;
        for (auto &s : e->slots) inflight += (int64_t)s->ids.size();
        out[0] = (int64_t)e->queue.size();
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
