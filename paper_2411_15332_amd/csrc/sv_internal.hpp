// Internal declarations shared by the C-ABI sources (handles, plan upload).
#pragma once

#include <exception>
#include <new>

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sv.h"
#include "sv_lower.hpp"
#include "sv_planner.hpp"

namespace sv {

sv_status fail(sv_status st, const char *fmt, ...);

// Runs an entry point's body so that no C++ exception crosses the C ABI: a
// failed host allocation is SV_ENOMEM, a broken internal invariant
// SV_EUNSUPPORTED (with the reason in sv_last_error).
template <class F>
sv_status guarded(F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(SV_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SV_EUNSUPPORTED, "internal error: %s", e.what());
    } catch (...) {
        return fail(SV_EUNSUPPORTED, "internal error");
    }
}
sv_status hip_fail(hipError_t e, const char *what);
size_t align_up(size_t x, size_t a);

#define SV_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return sv::hip_fail(e_, what); \
    } while (0)

}  // namespace sv

// A state handle (opaque to callers): state memory, stream, options, and the
// buffers used to upload pass plans.
struct sv_state_s {
    int n = 0;
    sv_dtype dt = SV_C128;
    int batch = 1;
    size_t amp_bytes = 16;
    size_t bytes = 0;
    void *buf = nullptr;
    bool owned = false;
    int device = 0;
    hipStream_t stream = nullptr;

    bool basis_known = true;
    uint64_t basis_j = 0;
    bool fill_pending = false;   // basis_j recorded but not yet written to the buffer

    // options
    bool fuse = true;
    int min_low = 0;      // 0: chosen per circuit (build_plan_auto)
    int max_dense = 1 << 20;
    bool gen_h = true;
    int small_mode = 1;
    bool remap = true;
    int pipeline = 0;   // SV_OPT_PIPELINE
    bool profile = false;

    // plan upload: pinned staging + device copy
    void *h_stage = nullptr;
    size_t h_cap = 0;
    void *d_plan = nullptr;
    size_t d_cap = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;

    // readout scratch
    double *d_red = nullptr;
    size_t d_red_cap = 0;
    double *h_out = nullptr;
    size_t h_out_cap = 0;
    uint64_t *d_idx = nullptr;
    size_t d_idx_cap = 0;

    // adjoint: work buffer of 2 * batch states (psi then lambda) and gradients
    void *d_work = nullptr;
    size_t d_work_cap = 0;
    double *d_grad = nullptr;
    size_t d_grad_cap = 0;

    // The last sv_apply_circuit plan, reused when the next call brings the
    // same gate records under the same plan options (starting basis state
    // included); only its constants are materialized again (parameters may
    // differ). Planning is host work; every pass still runs on the device.
    std::vector<sv_gate> plan_gates;
    size_t plan_nparams = 0;
    sv::PlanOptions plan_opts;
    sv::Lowering plan_low;   // the gates the plan was built from (composite kinds lowered)
    sv::Plan plan;
    bool plan_valid = false;
    // the device plan buffer holds `plan` serialized for dplan_batch entries
    // and this parameter table: a repeated sv_apply_circuit uploads nothing
    bool dplan_current = false;
    int dplan_batch = 0;
    std::vector<double> dplan_params;

    int64_t stats[8] = {0};

    struct Timed { hipEvent_t a, b; double bytes; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace sv {

PlanOptions plan_options(const sv_state_s *s);
sv_status ensure_device_buf(void **p, size_t *cap, size_t need, const char *what);
sv_status materialize(sv_state_s *s);
sv_status ensure_host_buf(void **p, size_t *cap, size_t need, const char *what);
// Upload plan `p` and launch it on `state` (`batch` states) on the handle's stream.
// uploaded: the device plan buffer already holds this serialization (the
// caller checked plan, batch and parameters); otherwise it is uploaded.
sv_status run_plan(sv_state_s *s, void *state, int batch, const Plan &p, const sv_gate *gates,
                   const double *params, size_t n_params, bool uploaded = false);
// Release every buffer the handle owns or caches (not the handle itself).
void release_handle_buffers(sv_state_s *s);

}  // namespace sv
