// C ABI of the state-vector library: handles, validation, errors, streams,
// plan upload and kernel launches. Declarations and contracts: include/sv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sv.h"
#include "../../include/sv_debug.h"
#include "sv_kernels.hpp"
#include "sv_planner.hpp"
#include "sv_internal.hpp"

using namespace sv;

namespace sv {

thread_local std::string g_err;

sv_status fail(sv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sv_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }




PlanOptions plan_options(const sv_state_s *s) {
    PlanOptions o;
    if (s->dt == SV_C128) {
        o.R = kRegBitsC128;
        o.v = 0;
        o.m = 3;
        o.small_max = kSmallMaxQubitsC128;
        o.ud_max = kMaxUdTermsC128;
    } else {
        o.R = kRegBitsC64;
        o.v = 1;
        o.m = 4;
        o.small_max = kSmallMaxQubitsC64;
        o.ud_max = kMaxUdTerms;
    }
    o.c = s->min_low ? s->min_low : 6;
    o.auto_low = s->min_low == 0;
    o.w_max = s->dt == SV_C128 ? kThreadBitsC128 : kThreadBitsC64;
    o.fuse = s->fuse;
    o.max_dense = s->max_dense;
    o.gen_h = s->gen_h;
    o.basis_known = s->basis_known;
    o.basis_j = s->basis_j;
    o.gen_basis = s->basis_known && s->fill_pending;
    o.small_mode = s->small_mode;
    o.remap = s->remap;
    return o;
}

// Write a recorded basis state into the buffer (sv_alloc and sv_set_basis
// only record it, so that the next circuit's first pass can generate it
// instead of reading a filled state).
sv_status materialize(sv_state_s *s) {
    if (!s->fill_pending) return SV_OK;
    SV_HIP(launch_fill_basis((int)s->dt, s->buf, 1ull << s->n, s->batch, s->basis_j, s->stream), "launch fill");
    s->fill_pending = false;
    return SV_OK;
}

sv_status ensure_device_buf(void **p, size_t *cap, size_t need, const char *what) {
    if (*cap >= need) return SV_OK;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return hip_fail(e, what);
    }
    size_t sz = std::max<size_t>(need, 4096);
    SV_HIP(hipMalloc(p, sz), what);
    *cap = sz;
    return SV_OK;
}

sv_status ensure_host_buf(void **p, size_t *cap, size_t need, const char *what) {
    if (*cap >= need) return SV_OK;
    if (*p) {
        hipError_t e = hipHostFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return hip_fail(e, what);
    }
    size_t sz = std::max<size_t>(need, 4096);
    SV_HIP(hipHostMalloc(p, sz, hipHostMallocDefault), what);
    *cap = sz;
    return SV_OK;
}

hipEvent_t get_event(sv_state_s *s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Sections of the uploaded plan, 256-byte aligned.
struct Layout {
    size_t passes = 0, layouts = 0, ops = 0, sops = 0, consts = 0, total = 0;
};

Layout plan_sections(const Plan &p, int batch, size_t real_bytes) {
    Layout L;
    size_t o = 0;
    L.passes = o;
    o = align_up(o + p.passes.size() * sizeof(DevPass), 256);
    L.layouts = o;
    o = align_up(o + p.layouts.size() * sizeof(DevLayout), 256);
    L.ops = o;
    o = align_up(o + (size_t)batch * p.ops.size() * sizeof(DevOp), 256);
    L.sops = o;
    o = align_up(o + p.sops.size() * sizeof(SmallOp), 256);
    L.consts = o;
    o = align_up(o + (size_t)batch * p.cstride * real_bytes, 256);
    L.total = std::max<size_t>(o, 256);
    return L;
}

void serialize_plan(const Plan &p, const Layout &L, const sv_gate *gates, const double *params,
                    size_t n_params, int batch, bool f32, char *dst) {
    if (!p.passes.empty()) std::memcpy(dst + L.passes, p.passes.data(), p.passes.size() * sizeof(DevPass));
    if (!p.layouts.empty())
        std::memcpy(dst + L.layouts, p.layouts.data(), p.layouts.size() * sizeof(DevLayout));
    if (!p.ops.empty()) materialize_ops(p, gates, params, n_params, batch, f32, dst + L.ops);
    if (!p.sops.empty()) std::memcpy(dst + L.sops, p.sops.data(), p.sops.size() * sizeof(SmallOp));
    if (p.cstride) materialize_consts(p, gates, params, n_params, batch, f32, dst + L.consts);
}

sv_status check_handle(sv_state s) {
    if (!s) return fail(SV_EINVAL, "null handle");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return SV_OK;
}

// Upload plan and launch it on the handle's stream, on `state`.
sv_status run_plan(sv_state_s *s, void *state, int batch, const Plan &p, const sv_gate *gates,
                   const double *params, size_t n_params, bool uploaded) {
    const bool f32 = s->dt == SV_C64;
    const size_t real_bytes = f32 ? 4 : 8;
    const Layout L = plan_sections(p, batch, real_bytes);
    if (!uploaded) {
        s->dplan_current = false;   // the upload below replaces what the buffer held
        if (s->upload_pending) {
            SV_HIP(hipEventSynchronize(s->upload_done), "wait for previous plan upload");
            s->upload_pending = false;
        }
        sv_status st = ensure_host_buf(&s->h_stage, &s->h_cap, L.total, "hipHostMalloc(plan)");
        if (st != SV_OK) return st;
        // the device plan buffer may still be read by queued kernels: grow only
        // after the stream has drained
        if (s->d_cap < L.total) {
            SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
            st = ensure_device_buf(&s->d_plan, &s->d_cap, L.total, "hipMalloc(plan)");
            if (st != SV_OK) return st;
        }
        serialize_plan(p, L, gates, params, n_params, batch, f32, static_cast<char *>(s->h_stage));
        SV_HIP(hipMemcpyAsync(s->d_plan, s->h_stage, L.total, hipMemcpyHostToDevice, s->stream),
               "hipMemcpyAsync(plan)");
        if (!s->upload_done) SV_HIP(hipEventCreateWithFlags(&s->upload_done, hipEventDisableTiming), "hipEventCreate");
        SV_HIP(hipEventRecord(s->upload_done, s->stream), "hipEventRecord");
        s->upload_pending = true;
    }

    char *d = static_cast<char *>(s->d_plan);
    const uint64_t N = 1ull << s->n;
    const double io_bytes = 2.0 * (double)N * (double)s->amp_bytes * batch;
    if (p.small) {
        if (p.sops.empty()) return SV_OK;
        hipEvent_t ea = nullptr, eb = nullptr;
        if (s->profile) {
            ea = get_event(s);
            eb = get_event(s);
            if (ea) hipEventRecord(ea, s->stream);
        }
        SV_HIP(launch_small((int)s->dt, state, s->n, batch,
                            reinterpret_cast<const SmallOp *>(d + L.sops), (int)p.sops.size(),
                            d + L.consts, p.cstride, s->stream),
               "launch k_small");
        if (s->profile && ea && eb) {
            hipEventRecord(eb, s->stream);
            s->timed.push_back({ea, eb, io_bytes});
        }
        return SV_OK;
    }
    const DevPass *dpass = reinterpret_cast<const DevPass *>(d + L.passes);
    for (size_t i = 0; i < p.passes.size(); ++i) {
        hipEvent_t ea = nullptr, eb = nullptr;
        if (s->profile) {
            ea = get_event(s);
            eb = get_event(s);
            if (ea) hipEventRecord(ea, s->stream);
        }
        SV_HIP(launch_pass((int)s->dt, state, N, batch, dpass, (int)i, p.passes[i],
                           reinterpret_cast<const DevLayout *>(d + L.layouts),
                           reinterpret_cast<const DevOp *>(d + L.ops), (uint64_t)p.ops.size(),
                           s->pipeline, s->stream),
               "launch k_pass");
        if (s->profile && ea && eb) {
            hipEventRecord(eb, s->stream);
            const bool gen = (p.passes[i].flags & PASS_GENERATES) != 0;
            s->timed.push_back({ea, eb, gen ? io_bytes * 0.5 : io_bytes});
        }
    }
    return SV_OK;
}

void release_handle_buffers(sv_state_s *s) {
    for (auto &t : s->timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    s->timed.clear();
    for (hipEvent_t ev : s->event_pool) hipEventDestroy(ev);
    s->event_pool.clear();
    if (s->upload_done) hipEventDestroy(s->upload_done);
    s->upload_done = nullptr;
    if (s->owned && s->buf) hipFree(s->buf);
    s->buf = nullptr;
    if (s->d_work) hipFree(s->d_work);
    if (s->d_grad) hipFree(s->d_grad);
    if (s->d_plan) hipFree(s->d_plan);
    if (s->d_red) hipFree(s->d_red);
    if (s->d_idx) hipFree(s->d_idx);
    if (s->h_stage) hipHostFree(s->h_stage);
    if (s->h_out) hipHostFree(s->h_out);
    s->d_work = nullptr;
    s->d_grad = nullptr;
    s->d_plan = nullptr;
    s->d_red = nullptr;
    s->d_idx = nullptr;
    s->h_stage = nullptr;
    s->h_out = nullptr;
}

int64_t plan_hbm_bytes(const Plan &p, int n, size_t amp_bytes) {
    const int64_t N = 1ll << n;
    if (p.small) return p.sops.empty() ? 0 : 2 * N * (int64_t)amp_bytes;
    int64_t b = 0;
    for (const DevPass &dp : p.passes)
        b += ((dp.flags & PASS_GENERATES) ? 1 : 2) * N * (int64_t)amp_bytes;
    return b;
}

}  // namespace sv

extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

const char *sv_version(void) { return "sv-gfx950 0.1"; }

sv_status sv_alloc(int n_qubits, sv_dtype dtype, int batch, void *dev_buf, size_t buf_bytes,
                   void *hip_stream, sv_state *out) {
    return guarded([&]() -> sv_status {
        if (!out) return fail(SV_EINVAL, "out is NULL");
        *out = nullptr;
        if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d outside 1..34", n_qubits);
        if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "unknown dtype %d", (int)dtype);
        if (batch < 1 || batch > 65535) return fail(SV_EINVAL, "batch %d outside 1..65535", batch);
        const size_t amp = dtype == SV_C128 ? 16 : 8;
        const size_t bytes = ((size_t)1 << n_qubits) * amp * (size_t)batch;
        if (dev_buf) {
            if (buf_bytes < bytes)
                return fail(SV_EINVAL, "buffer of %zu bytes is smaller than the %zu needed", buf_bytes, bytes);
            if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0)
                return fail(SV_EINVAL, "device buffer is not 256-byte aligned");
        }
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        sv_state_s *s = new (std::nothrow) sv_state_s();
        if (!s) return fail(SV_ENOMEM, "host allocation failed");
        s->n = n_qubits;
        s->dt = dtype;
        s->batch = batch;
        s->amp_bytes = amp;
        s->bytes = bytes;
        s->device = dev;
        s->stream = static_cast<hipStream_t>(hip_stream);
        if (const char *fail_alloc = std::getenv("SV_DEBUG_FAIL_ALLOC")) {
            if (std::atoi(fail_alloc) != 0 && !dev_buf) {
                delete s;
                return fail(SV_ENOMEM, "allocation failure injected by SV_DEBUG_FAIL_ALLOC");
            }
        }
        if (dev_buf) {
            s->buf = dev_buf;
            s->owned = false;
        } else {
            e = hipMalloc(&s->buf, bytes);
            if (e != hipSuccess) {
                delete s;
                return hip_fail(e, "hipMalloc(state)");
            }
            s->owned = true;
        }
        // |0...0> is written by the first pass of the first circuit (generated,
        // not read) or by materialize() before anything else reads the buffer
        s->basis_known = true;
        s->basis_j = 0;
        s->fill_pending = true;
        *out = s;
        return SV_OK;
    });
}

sv_status sv_free(sv_state s) {
    return guarded([&]() -> sv_status {
        if (!s) return SV_OK;
        hipSetDevice(s->device);
        hipError_t e = hipStreamSynchronize(s->stream);
        release_handle_buffers(s);
        delete s;
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize at free");
        return SV_OK;
    });
}

sv_status sv_set_stream(sv_state s, void *hip_stream) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        s->stream = static_cast<hipStream_t>(hip_stream);
        return SV_OK;
    });
}

sv_status sv_set_basis(sv_state s, uint64_t j) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (j >= (1ull << s->n)) return fail(SV_EINVAL, "basis index %llu >= 2^%d", (unsigned long long)j, s->n);
        s->basis_known = true;
        s->basis_j = j;
        s->fill_pending = true;
        return SV_OK;
    });
}

sv_status sv_mark_modified(sv_state s) {
    return guarded([&]() -> sv_status {
        if (!s) return fail(SV_EINVAL, "null handle");
        s->basis_known = false;
        s->fill_pending = false;
        return SV_OK;
    });
}

sv_status sv_apply_circuit(sv_state s, const sv_gate *gates, size_t n_gates, const double *params,
                           size_t n_params) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (n_gates && !gates) return fail(SV_EINVAL, "gates is NULL");
        std::string err;
        if (!validate_gates(s->n, gates, n_gates, n_params, params != nullptr, err))
            return fail(SV_EINVAL, "%s", err.c_str());
        if (n_gates == 0) return SV_OK;
        const PlanOptions po = plan_options(s);
        const bool hit = s->plan_valid && s->plan_gates.size() == n_gates && s->plan_nparams == n_params &&
                         same_options(s->plan_opts, po) &&
                         std::memcmp(s->plan_gates.data(), gates, n_gates * sizeof(sv_gate)) == 0;
        if (!hit) {
            s->plan_valid = false;
            s->dplan_current = false;
            lower_gates(gates, n_gates, n_params, s->plan_low);
            s->plan = build_plan_auto(s->n, s->plan_low.gates.data(), s->plan_low.gates.size(), po);
            s->plan_gates.assign(gates, gates + n_gates);
            s->plan_nparams = n_params;
            s->plan_opts = po;
            s->plan_valid = true;
        }
        const Plan &p = s->plan;
        if (s->fill_pending && (p.small || p.passes.empty() || !(p.passes[0].flags & PASS_GENERATES))) {
            st = materialize(s);   // this plan reads its input
            if (st != SV_OK) return st;
        }
        std::vector<double> ext;
        lower_params(s->plan_low, params, n_params, s->batch, ext);
        const double *pp = ext.empty() ? params : ext.data();
        const size_t np = ext.empty() ? n_params : n_params + s->plan_low.src.size();
        const size_t cnt = pp ? np * (size_t)s->batch : 0;
        // the same plan, batch and parameters as the last upload: the device
        // plan buffer already holds this serialization
        const bool same = s->dplan_current && s->dplan_batch == s->batch && s->dplan_params.size() == cnt &&
                          (cnt == 0 || std::memcmp(s->dplan_params.data(), pp, cnt * sizeof(double)) == 0);
        st = run_plan(s, s->buf, s->batch, p, s->plan_low.gates.data(), pp, np, same);
        if (st != SV_OK) return st;
        if (!same) {
            s->dplan_current = true;
            s->dplan_batch = s->batch;
            s->dplan_params.assign(pp, pp + cnt);
        }
        s->fill_pending = false;   // the first pass generated the recorded basis state
        s->stats[0] = p.small ? 1 : (int64_t)p.passes.size();
        s->stats[1] = p.n_exch;
        s->stats[2] = p.gates_applied;
        s->stats[3] = p.n_gen_h;
        s->stats[4] = p.small ? (p.sops.empty() ? 0 : 1) : (int64_t)p.passes.size();
        s->stats[5] = plan_hbm_bytes(p, s->n, s->amp_bytes);
        s->stats[6] = p.n_relabel;
        s->stats[7] = p.n_gen_product;
        if (p.gates_applied > 0) s->basis_known = false;
        return SV_OK;
    });
}

static sv_status reduce(sv_state s, int qubit, double *out) {
    sv_status st0 = materialize(s);
    if (st0 != SV_OK) return st0;
    const size_t np = reduce_partials_size(s->n) * (size_t)s->batch + (size_t)s->batch;
    sv_status st = ensure_device_buf(reinterpret_cast<void **>(&s->d_red), &s->d_red_cap,
                                     np * sizeof(double), "hipMalloc(reduce)");
    if (st != SV_OK) return st;
    st = ensure_host_buf(reinterpret_cast<void **>(&s->h_out), &s->h_out_cap,
                         (size_t)s->batch * sizeof(double), "hipHostMalloc(out)");
    if (st != SV_OK) return st;
    double *d_out = s->d_red + reduce_partials_size(s->n) * (size_t)s->batch;
    SV_HIP(launch_reduce((int)s->dt, s->buf, s->n, s->batch, qubit, s->d_red, d_out, s->stream),
           "launch reduce");
    SV_HIP(hipMemcpyAsync(s->h_out, d_out, (size_t)s->batch * sizeof(double), hipMemcpyDeviceToHost,
                          s->stream),
           "hipMemcpyAsync(out)");
    SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    std::memcpy(out, s->h_out, (size_t)s->batch * sizeof(double));
    return SV_OK;
}

sv_status sv_expect_z(sv_state s, int qubit, double *out) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (!out) return fail(SV_EINVAL, "out is NULL");
        if (qubit < 0 || qubit >= s->n) return fail(SV_EINVAL, "qubit %d out of range for n = %d", qubit, s->n);
        return reduce(s, qubit, out);
    });
}

sv_status sv_norm(sv_state s, double *out) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (!out) return fail(SV_EINVAL, "out is NULL");
        return reduce(s, -1, out);
    });
}

sv_status sv_expect_z_noalloc(const void *state, int n_qubits, sv_dtype dtype, int batch, int qubit,
                              double *out, void *hip_stream) {
    return guarded([&]() -> sv_status {
        // every argument is checked before any HIP call, so a rejected call
        // launches nothing and leaves the scratch as it was
        if (!state || !out) return fail(SV_EINVAL, "state or out is NULL");
        if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "unknown dtype %d", (int)dtype);
        if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d outside 1..34", n_qubits);
        if (batch < 1 || batch > 65535) return fail(SV_EINVAL, "batch %d outside 1..65535", batch);
        if (qubit < -1 || qubit >= n_qubits)
            return fail(SV_EINVAL, "qubit %d out of range for n = %d", qubit, n_qubits);
        // 16-byte loads in both precisions (two complex64 amplitudes at a time)
        if (reinterpret_cast<uintptr_t>(state) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 8 != 0)
            return fail(SV_EINVAL, "state or out is misaligned");
        const size_t need = reduce_partials_size(n_qubits) * (size_t)batch;
        if (need > kStaticPartials)
            return fail(SV_EINVAL, "batch %d of n = %d needs %zu partial sums; the static scratch holds %zu",
                        batch, n_qubits, need, kStaticPartials);
        double *part = nullptr;
        SV_HIP(static_partials(&part), "scratch address");
        SV_HIP(launch_reduce((int)dtype, state, n_qubits, batch, qubit, part, out,
                             static_cast<hipStream_t>(hip_stream)),
               "launch reduce");
        return SV_OK;
    });
}

sv_status sv_amplitudes(sv_state s, int b, const uint64_t *idx, size_t k, double *out) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (b < 0 || b >= s->batch) return fail(SV_EINVAL, "batch entry %d out of range", b);
        if (k == 0) return SV_OK;
        if (!idx || !out) return fail(SV_EINVAL, "idx or out is NULL");
        const uint64_t N = 1ull << s->n;
        for (size_t i = 0; i < k; ++i)
            if (idx[i] >= N) return fail(SV_EINVAL, "index %llu >= 2^%d", (unsigned long long)idx[i], s->n);
        st = materialize(s);
        if (st != SV_OK) return st;
        const size_t need_host = std::max(k * sizeof(uint64_t), 2 * k * sizeof(double));
        st = ensure_host_buf(reinterpret_cast<void **>(&s->h_out), &s->h_out_cap, need_host, "hipHostMalloc");
        if (st != SV_OK) return st;
        st = ensure_device_buf(reinterpret_cast<void **>(&s->d_idx), &s->d_idx_cap,
                               k * sizeof(uint64_t) + 2 * k * sizeof(double), "hipMalloc(idx)");
        if (st != SV_OK) return st;
        // the pinned buffer may still feed an earlier copy only after a sync, which
        // every readout performs; safe to reuse here
        std::memcpy(s->h_out, idx, k * sizeof(uint64_t));
        SV_HIP(hipMemcpyAsync(s->d_idx, s->h_out, k * sizeof(uint64_t), hipMemcpyHostToDevice, s->stream),
               "hipMemcpyAsync(idx)");
        double *d_vals = reinterpret_cast<double *>(s->d_idx + k);
        const char *base = static_cast<const char *>(s->buf) + (size_t)b * N * s->amp_bytes;
        SV_HIP(launch_gather((int)s->dt, base, s->d_idx, k, d_vals, s->stream), "launch gather");
        SV_HIP(hipMemcpyAsync(s->h_out, d_vals, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s->stream),
               "hipMemcpyAsync(amplitudes)");
        SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        std::memcpy(out, s->h_out, 2 * k * sizeof(double));
        return SV_OK;
    });
}

sv_status sv_sync(sv_state s) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        st = materialize(s);
        if (st != SV_OK) return st;
        SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        return SV_OK;
    });
}

void *sv_device_ptr(sv_state s) {
    if (!s) return nullptr;
    try {
        materialize(s);   // a failed launch surfaces at the next synchronizing call
    } catch (...) {
    }
    return s->buf;
}

sv_status sv_set_option(sv_state s, int option, int64_t value) {
    return guarded([&]() -> sv_status {
        if (!s) return fail(SV_EINVAL, "null handle");
        switch (option) {
        case SV_OPT_FUSE:
            if (value != 0 && value != 1) return fail(SV_EINVAL, "SV_OPT_FUSE takes 0 or 1");
            s->fuse = value != 0;
            return SV_OK;
        case SV_OPT_MIN_LOW_QUBITS:
            if (value != 0 && (value < 3 || value > 7))
                return fail(SV_EINVAL, "SV_OPT_MIN_LOW_QUBITS takes 0 (automatic) or 3..7");
            s->min_low = (int)value;
            return SV_OK;
        case SV_OPT_MAX_DENSE:
            if (value < 1 || value > (1 << 20)) return fail(SV_EINVAL, "SV_OPT_MAX_DENSE takes >= 1");
            s->max_dense = (int)value;
            return SV_OK;
        case SV_OPT_ON_DEMAND_H:
            if (value != 0 && value != 1) return fail(SV_EINVAL, "SV_OPT_ON_DEMAND_H takes 0 or 1");
            s->gen_h = value != 0;
            return SV_OK;
        case SV_OPT_SMALL_PATH:
            if (value != 1 && value != 2) return fail(SV_EINVAL, "SV_OPT_SMALL_PATH takes 1 or 2");
            s->small_mode = (int)value;
            return SV_OK;
        case SV_OPT_PROFILE:
            if (value != 0 && value != 1) return fail(SV_EINVAL, "SV_OPT_PROFILE takes 0 or 1");
            s->profile = value != 0;
            return SV_OK;
        case SV_OPT_REMAP:
            if (value != 0 && value != 1) return fail(SV_EINVAL, "SV_OPT_REMAP takes 0 or 1");
            s->remap = value != 0;
            return SV_OK;
        case SV_OPT_PIPELINE:
            if (value < 0 || value > 2) return fail(SV_EINVAL, "SV_OPT_PIPELINE takes 0, 1 or 2");
            s->pipeline = (int)value;
            return SV_OK;
        default:
            return fail(SV_EINVAL, "unknown option %d", option);
        }
    });
}

sv_status sv_plan_stats(sv_state s, int64_t out[8]) {
    return guarded([&]() -> sv_status {
        if (!s || !out) return fail(SV_EINVAL, "null argument");
        std::memcpy(out, s->stats, sizeof s->stats);
        return SV_OK;
    });
}

sv_status sv_profile_read(sv_state s, double *total_ms, int64_t *launches, double *bytes) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        double tot = 0.0, by = 0.0;
        for (auto &t : s->timed) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, t.a, t.b);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            tot += ms;
            by += t.bytes;
            s->event_pool.push_back(t.a);
            s->event_pool.push_back(t.b);
        }
        if (total_ms) *total_ms = tot;
        if (launches) *launches = (int64_t)s->timed.size();
        if (bytes) *bytes = by;
        s->timed.clear();
        return SV_OK;
    });
}

sv_status sv_adjoint_expect_z(sv_state s, const sv_gate *gates, size_t n_gates, const double *params,
                              size_t n_params, int qubit, double *expect, double *grad) {
    return guarded([&]() -> sv_status {
        sv_status st = check_handle(s);
        if (st != SV_OK) return st;
        if (qubit < 0 || qubit >= s->n) return fail(SV_EINVAL, "qubit %d out of range for n = %d", qubit, s->n);
        if (n_gates && !gates) return fail(SV_EINVAL, "gates is NULL");
        if (n_params && !grad) return fail(SV_EINVAL, "grad is NULL");
        std::string err;
        if (!validate_gates(s->n, gates, n_gates, n_params, params != nullptr, err))
            return fail(SV_EINVAL, "%s", err.c_str());
        for (size_t i = 0; i < n_gates; ++i) {
            const int k = gates[i].kind;
            if (gates[i].param >= 0 && k != SV_GATE_RX && k != SV_GATE_RY && k != SV_GATE_RZ)
                return fail(SV_EUNSUPPORTED, "gate %zu: only RX, RY and RZ may reference parameters", i);
        }
        // composite kinds (fixed angles only, checked above) become planner
        // kinds; every parametric gate keeps its parameter index
        Lowering low;
        lower_gates(gates, n_gates, n_params, low);
        gates = low.gates.data();
        n_gates = low.gates.size();
        const int B = s->batch;
        const uint64_t N = 1ull << s->n;
        const size_t state_bytes = (size_t)N * s->amp_bytes;
        st = ensure_device_buf(&s->d_work, &s->d_work_cap, 2 * (size_t)B * state_bytes, "hipMalloc(adjoint work)");
        if (st != SV_OK) return st;
        const size_t ngrad = std::max<size_t>(1, (size_t)B * n_params);
        st = ensure_device_buf(reinterpret_cast<void **>(&s->d_grad), &s->d_grad_cap,
                               ngrad * sizeof(double), "hipMalloc(grad)");
        if (st != SV_OK) return st;
        // partials: reductions (batch + 1 rows) and up to kMaxIpTerms fused inner products
        const size_t np = pauli_ip_partials_size(s->n) * (size_t)B * kMaxIpTerms + (size_t)B;
        st = ensure_device_buf(reinterpret_cast<void **>(&s->d_red), &s->d_red_cap, np * sizeof(double),
                               "hipMalloc(reduce)");
        if (st != SV_OK) return st;
        const int chunk_bits = pauli_ip_multi_chunk_bits(s->n);
        char *psi = static_cast<char *>(s->d_work);
        char *lam = psi + (size_t)B * state_bytes;
        const int dt = (int)s->dt;

        // forward: psi = U |0...0> for every batch entry (generated by the
        // first pass when the plan has passes, else filled first)
        PlanOptions po = plan_options(s);
        po.basis_known = true;
        po.basis_j = 0;
        po.gen_basis = true;
        {
            Plan p = build_plan(s->n, gates, n_gates, po);
            if (p.small || p.passes.empty() || !(p.passes[0].flags & PASS_GENERATES))
                SV_HIP(launch_fill_basis(dt, psi, N, B, 0, s->stream), "launch fill");
            st = run_plan(s, psi, B, p, gates, params, n_params);
            if (st != SV_OK) return st;
        }
        SV_HIP(hipMemcpyAsync(s->buf, psi, (size_t)B * state_bytes, hipMemcpyDeviceToDevice, s->stream),
               "hipMemcpyAsync(final states)");
        s->basis_known = false;
        s->fill_pending = false;
        // f = <Z_q> and lambda = Z_q psi
        double *d_out = s->d_red + reduce_partials_size(s->n) * (size_t)B;
        SV_HIP(launch_reduce(dt, psi, s->n, B, qubit, s->d_red, d_out, s->stream), "launch reduce");
        if (expect) {
            st = ensure_host_buf(reinterpret_cast<void **>(&s->h_out), &s->h_out_cap, (size_t)B * sizeof(double),
                                 "hipHostMalloc(out)");
            if (st != SV_OK) return st;
            SV_HIP(hipMemcpyAsync(s->h_out, d_out, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, s->stream),
                   "hipMemcpyAsync(expect)");
            SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
            std::memcpy(expect, s->h_out, (size_t)B * sizeof(double));
        }
        SV_HIP(launch_copy_z(dt, psi, lam, N, B, qubit, s->stream), "launch copy_z");
        SV_HIP(hipMemsetAsync(s->d_grad, 0, ngrad * sizeof(double), s->stream), "hipMemsetAsync(grad)");

        // reverse sweep on the 2B states [psi | lambda] with the inverse gates;
        // parameter rows are duplicated and negated (U(t)^dagger = U(-t) for rotations)
        std::vector<double> pneg((size_t)2 * B * std::max<size_t>(n_params, 1), 0.0);
        for (int b = 0; b < B; ++b)
            for (size_t p = 0; p < n_params; ++p) {
                pneg[(size_t)b * n_params + p] = -params[(size_t)b * n_params + p];
                pneg[(size_t)(B + b) * n_params + p] = -params[(size_t)b * n_params + p];
            }
        auto inverse = [](sv_gate g) {
            switch (g.kind) {
            case SV_GATE_S: g.kind = SV_GATE_SDG; break;
            case SV_GATE_SDG: g.kind = SV_GATE_S; break;
            case SV_GATE_T: g.kind = SV_GATE_TDG; break;
            case SV_GATE_TDG: g.kind = SV_GATE_T; break;
            case SV_GATE_RX: case SV_GATE_RY: case SV_GATE_RZ: case SV_GATE_P: case SV_GATE_CPHASE:
                if (g.param < 0) g.angle = -g.angle;   // referenced angles come from the negated table
                break;
            default: break;   // X, Y, Z, H, CNOT, CZ, SWAP, CCX, MARK, I are self-inverse
            }
            return g;
        };
        PlanOptions pr = plan_options(s);
        pr.basis_known = false;
        std::vector<sv_gate> seg;
        auto flush = [&]() -> sv_status {
            if (seg.empty()) return SV_OK;
            Plan p = build_plan(s->n, seg.data(), seg.size(), pr);
            sv_status r = run_plan(s, psi, 2 * B, p, seg.data(), pneg.data(), n_params);
            seg.clear();
            return r;
        };
        // A run of consecutive parametric rotations on distinct qubits shares
        // one state pair: the generator of each (a Pauli on its own qubit)
        // commutes with the run's later rotations, so <lambda_k| P_k |psi_k>
        // equals <lambda| P_k |psi> taken after the run's last gate, and the
        // whole run is then undone in one segment.
        // A diagonal unitary D applied to both states leaves every Z term
        // unchanged (<D lambda| Z_q |D psi> = <lambda| Z_q |psi>: D commutes
        // with Z_q and D^dagger D = I). So Z terms wait while only diagonal
        // gates are undone, and join the next run's read of the states; any
        // other gate to undo first sends them out at the point they belong to.
        auto diagonal = [](const sv_gate &g) {
            switch (g.kind) {
            case SV_GATE_I: case SV_GATE_Z: case SV_GATE_S: case SV_GATE_SDG: case SV_GATE_T:
            case SV_GATE_TDG: case SV_GATE_RZ: case SV_GATE_P: case SV_GATE_CZ: case SV_GATE_CPHASE:
            case SV_GATE_MARK: case SV_GATE_CRZ: case SV_GATE_RZZ: case SV_GATE_CU1:
                return true;
            default:
                return false;
            }
        };
        struct ZTerm {
            uint8_t q;
            uint64_t off;
        };
        std::vector<ZTerm> pend_z;   // Z terms still valid at the current point
        bool seg_diag = true;        // every gate queued in seg is diagonal
        // Launch the contiguous-chunk inner products of `zs` (Z terms) and
        // `xy` (X / Y terms on qubits below chunk_bits, at most kIpMaxXYTerms
        // of them) at the current point, kMaxIpTerms at a time.
        auto launch_low = [&](const std::vector<ZTerm> &zs, const std::vector<std::pair<sv_gate, int>> &xy)
            -> sv_status {
            IpTerms terms{};
            IpOffsets offs{};
            int nt = 0, nxy = 0;
            auto go = [&]() -> sv_status {
                if (nt) {
                    SV_HIP(launch_pauli_ip_multi(dt, psi, lam, s->n, B, terms, offs, nt, s->d_red, s->d_grad,
                                                 n_params, s->stream),
                           "launch pauli_ip_multi");
                }
                terms = IpTerms{};
                offs = IpOffsets{};
                nt = nxy = 0;
                return SV_OK;
            };
            for (const auto &t : xy) {
                if (nt == kMaxIpTerms || nxy == kIpMaxXYTerms) {
                    sv_status r = go();
                    if (r != SV_OK) return r;
                }
                terms.q[nt] = (uint8_t)t.first.q0;
                terms.pauli[nt] = (uint8_t)t.second;
                offs.off[nt] = (uint64_t)t.first.param;
                ++nt;
                ++nxy;
            }
            for (const ZTerm &z : zs) {
                if (nt == kMaxIpTerms) {
                    sv_status r = go();
                    if (r != SV_OK) return r;
                }
                terms.q[nt] = z.q;
                terms.pauli[nt] = 3;
                offs.off[nt] = z.off;
                ++nt;
            }
            return go();
        };
        size_t i = n_gates;
        while (i > 0) {
            const sv_gate &g = gates[i - 1];
            if (g.param < 0) {
                seg.push_back(inverse(g));
                seg_diag = seg_diag && diagonal(g);
                --i;
                continue;
            }
            size_t j = i;   // the run is gates[j .. i - 1]
            uint64_t used = 0;
            while (j > 0 && gates[j - 1].param >= 0 && !((used >> gates[j - 1].q0) & 1)) {
                used |= 1ull << gates[j - 1].q0;
                --j;
            }
            // Z terms waiting from later runs are still valid here if every
            // gate queued for undoing is diagonal; otherwise they go out now,
            // at the point they were taken, before that undo
            if (!pend_z.empty() && !seg_diag) {
                st = launch_low(pend_z, {});
                if (st != SV_OK) return st;
                pend_z.clear();
            }
            bool run_diag = true;   // this run's own undo is diagonal (RZ only)
            for (size_t k = j; k < i; ++k) run_diag = run_diag && gates[k].kind == SV_GATE_RZ;
            // An RZ-only run's terms all wait, so the states are not needed
            // at its own point. When only diagonal gates separate it from the
            // previous run, its undo joins the next segment instead of being
            // applied here: its terms, and those already waiting, are still
            // valid at that run's point and go with its launch.
            if (run_diag) {
                size_t k = j;
                while (k > 0 && gates[k - 1].param < 0 && diagonal(gates[k - 1])) --k;
                if (k > 0 && gates[k - 1].param >= 0) {
                    for (size_t t = i; t-- > j;)
                        pend_z.push_back(ZTerm{(uint8_t)gates[t].q0, (uint64_t)gates[t].param});
                    for (size_t t = i; t-- > j;) seg.push_back(inverse(gates[t]));
                    seg_diag = true;   // every waiting term stays valid through the next flush
                    i = j;
                    continue;
                }
            }
            st = flush();
            if (st != SV_OK) return st;
            // one read of psi and lambda for every Z term and every X / Y term
            // whose partner amplitude lies in the same 2^12-amplitude chunk;
            // one more read per group of up to 8 X / Y terms on higher qubits
            // (the run's qubits are distinct, so a group is up to 8 qubits)
            std::vector<ZTerm> zs;
            zs.swap(pend_z);
            std::vector<std::pair<sv_gate, int>> xy;
            std::vector<size_t> high;   // gate indices of X / Y terms on qubits >= chunk_bits
            for (size_t k = i; k-- > j;) {
                const sv_gate &gk = gates[k];
                const int pauli = gk.kind == SV_GATE_RX ? 1 : gk.kind == SV_GATE_RY ? 2 : 3;
                if (pauli == 3)
                    (run_diag ? pend_z : zs).push_back(ZTerm{(uint8_t)gk.q0, (uint64_t)gk.param});
                else if (gk.q0 < chunk_bits)
                    xy.emplace_back(gk, pauli);
                else
                    high.push_back(k);
            }
            st = launch_low(zs, xy);
            if (st != SV_OK) return st;
            for (size_t g0 = 0; g0 < high.size(); g0 += 8) {
                const size_t g1 = std::min(high.size(), g0 + 8);
                std::vector<int> qs;
                for (size_t t = g0; t < g1; ++t) qs.push_back(gates[high[t]].q0);
                std::sort(qs.begin(), qs.end());
                IpHiMap map{};
                map.h = (int32_t)qs.size();
                for (int k = 0; k < map.h; ++k) map.hq[k] = (uint8_t)qs[(size_t)k];
                IpTerms ht{};
                IpOffsets ho{};
                int hn = 0;
                for (size_t t = g0; t < g1; ++t) {
                    const sv_gate &gk = gates[high[t]];
                    const int pos = (int)(std::lower_bound(qs.begin(), qs.end(), (int)gk.q0) - qs.begin());
                    ht.q[hn] = (uint8_t)(12 - map.h + pos);   // the qubit's bit inside the staged sub-chunk
                    ht.pauli[hn] = (uint8_t)(gk.kind == SV_GATE_RX ? 1 : 2);
                    ho.off[hn] = (uint64_t)gk.param;
                    ++hn;
                }
                SV_HIP(launch_pauli_ip_hi(dt, psi, lam, s->n, B, ht, ho, hn, map, s->d_red, s->d_grad, n_params,
                                          s->stream),
                       "launch pauli_ip_hi");
            }
            for (size_t k = i; k-- > j;) seg.push_back(inverse(gates[k]));
            seg_diag = run_diag;
            i = j;
        }
        // Z terms still waiting are valid at the current point (the queued
        // undo has not been applied); that undo itself is never read
        st = launch_low(pend_z, {});
        if (st != SV_OK) return st;
        seg.clear();
        if (n_params) {
            std::vector<double> tmp((size_t)B * n_params);
            SV_HIP(hipMemcpyAsync(tmp.data(), s->d_grad, tmp.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream),
                   "hipMemcpyAsync(grad)");
            SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
            std::memcpy(grad, tmp.data(), tmp.size() * sizeof(double));
        } else {
            SV_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        }
        return SV_OK;
    });
}

// ---------------------------------------------------------------------------
// Diagnostics (include/sv_debug.h)

static int64_t debug_plan_impl(int n, int dtype, const sv_gate *gates, size_t n_gates,
                               const double *params, size_t n_params, const int64_t *opts,
                               void *out, size_t cap);

int64_t sv_debug_plan(int n, int dtype, const sv_gate *gates, size_t n_gates, const double *params,
                      size_t n_params, const int64_t *opts, void *out, size_t cap) {
    int64_t r = 0;
    const sv_status st = guarded([&]() -> sv_status {
        r = debug_plan_impl(n, dtype, gates, n_gates, params, n_params, opts, out, cap);
        return SV_OK;
    });
    return st == SV_OK ? r : (int64_t)st;
}

static int64_t debug_plan_impl(int n, int dtype, const sv_gate *gates, size_t n_gates,
                               const double *params, size_t n_params, const int64_t *opts,
                               void *out, size_t cap) {
    if (n < 1 || n > 34 || (dtype != SV_C64 && dtype != SV_C128)) {
        fail(SV_EINVAL, "bad n or dtype");
        return SV_EINVAL;
    }
    std::string err;
    if (!validate_gates(n, gates, n_gates, n_params, params != nullptr, err)) {
        fail(SV_EINVAL, "%s", err.c_str());
        return SV_EINVAL;
    }
    sv_state_s tmp;
    tmp.n = n;
    tmp.dt = (sv_dtype)dtype;
    if (opts) {
        tmp.fuse = opts[0] != 0;
        tmp.min_low = (int)opts[1];
        tmp.max_dense = (int)opts[2];
        tmp.gen_h = opts[3] != 0;
        tmp.basis_known = opts[4] != 0;
        tmp.basis_j = (uint64_t)opts[5];
        tmp.small_mode = (int)opts[6];
        tmp.remap = opts[7] != 0;
        tmp.fill_pending = opts[8] != 0;
    } else {
        tmp.fill_pending = false;
    }
    const PlanOptions po = plan_options(&tmp);
    Lowering low;
    lower_gates(gates, n_gates, n_params, low);
    std::vector<double> ext;
    lower_params(low, params, n_params, 1, ext);
    if (!ext.empty()) {
        params = ext.data();
        n_params += low.src.size();
    }
    gates = low.gates.data();
    n_gates = low.gates.size();
    Plan p = build_plan_auto(n, gates, n_gates, po);
    const size_t real_bytes = dtype == SV_C64 ? 4 : 8;  // constants in the state's precision
    const Layout L = plan_sections(p, 1, real_bytes);
    const size_t header = 256;
    const size_t total = header + L.total;
    if (!out || cap < total) return (int64_t)total;
    char *o = static_cast<char *>(out);
    std::memset(o, 0, total);
    int64_t *h = reinterpret_cast<int64_t *>(o);
    int k = 0, w = 0;
    tile_geometry(n, po, k, w);
    h[0] = p.small;
    h[1] = (int64_t)p.passes.size();
    h[2] = (int64_t)p.layouts.size();
    h[3] = (int64_t)p.ops.size();
    h[4] = (int64_t)p.sops.size();
    h[5] = (int64_t)p.cstride;
    h[6] = p.n_exch;
    h[7] = p.n_gen_h;
    h[8] = p.gates_applied;
    h[9] = k;
    h[10] = w;
    h[11] = po.R;
    h[12] = po.m;
    h[13] = (int64_t)(header + L.passes);
    h[14] = (int64_t)(header + L.layouts);
    h[15] = (int64_t)(header + L.ops);
    h[16] = (int64_t)(header + L.sops);
    h[17] = (int64_t)(header + L.consts);
    h[18] = plan_hbm_bytes(p, n, dtype == SV_C128 ? 16 : 8);
    h[19] = p.n_relabel;
    h[20] = p.n_restore;
    h[21] = p.low;
    h[22] = p.n_gen_product;
    serialize_plan(p, L, gates, params, n_params, 1, dtype == SV_C64, o + header);
    return (int64_t)total;
}

}  // extern "C"
