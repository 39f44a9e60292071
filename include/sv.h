/*
 * sv.h — C ABI of the MI355X (gfx950) state-vector gate-application library.
 *
 * The library applies the gates of a circuit in place to 2^n complex
 * amplitudes on one GPU, never forming the 2^n x 2^n operation matrix
 * U = I^(k-1) (x) G (x) I^(n-k) of the paper's Sec. II-A. Sparse gates are
 * applied from a gate-local compressed form (value + index, the DAX idea of
 * Sec. III-A), dense 1- and 2-qubit gates as strided butterflies, and
 * Hadamard layers from the RH rule of Sec. III-B (one magnitude 2^(-m/2) and
 * signs (-1)^popcount(r & c) computed on demand).
 *
 * Conventions
 *   - Amplitude index i = sum_q b_q 2^q: qubit q is bit q (the paper's qubit k,
 *     the k-th Kronecker factor from the left, is q = n - k).
 *   - A state is interleaved complex: SV_C128 = (double re, double im),
 *     SV_C64 = (float re, float im), the memory layout of torch.complex128 /
 *     torch.complex64. A batch of B states is [B][2^n], row-major.
 *   - A 2-qubit gate's 4x4 matrix is indexed by (b_q0 << 1) | b_q1: the first
 *     operand is the high local bit (CNOT: q0 = control, q1 = target).
 *
 * Errors
 *   Every call returns an sv_status and never throws. Argument errors are
 *   detected on the host before anything is launched and leave the state
 *   unchanged; sv_last_error() (thread-local) describes the last failure.
 *   Device faults surface as SV_EDEVICE at the next synchronizing call.
 *   A handle is not thread-safe: use it from one host thread.
 *
 * Streams
 *   All device work of a handle goes to the HIP stream given at sv_alloc
 *   (NULL = the default stream) or set later with sv_set_stream.
 *   sv_apply_circuit is asynchronous; the readouts synchronize that stream.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sv_status {
    SV_OK = 0,
    SV_EINVAL = -1,       /* bad argument: nothing was launched */
    SV_ENOMEM = -2,       /* device or host allocation failed */
    SV_EDEVICE = -3,      /* a HIP call or a kernel failed */
    SV_EUNSUPPORTED = -4  /* valid request this build does not support */
} sv_status;

typedef enum sv_dtype { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

/* Gate kinds. Matrices (c = cos(t/2), s = sin(t/2)):
 *   X = [[0,1],[1,0]], Y = [[0,-i],[i,0]] (both printed in Sec. III-A1),
 *   Z = diag(1,-1), H = [[1,1],[1,-1]]/sqrt2, S = diag(1,i), SDG = S^dagger,
 *   T = diag(1,e^{i pi/4}), TDG = T^dagger, RX(t) = [[c,-is],[-is,c]],
 *   RY(t) = [[c,-s],[s,c]], RZ(t) = diag(e^{-it/2}, e^{it/2}), P(t) = diag(1,e^{it}),
 *   CNOT, CZ = diag(1,1,1,-1), SWAP, CPHASE(t) = diag(1,1,1,e^{it}),
 *   MARK = I - 2|m><m| on all n qubits (m = sv_gate.index; the Grover oracle
 *   of Sec. IV-D, and with m = 0 the zero-state reflection),
 *   U1 / U2 = a general 2x2 / 4x4 complex matrix (any 1- or 2-qubit gate of
 *   Table 1), read from the parameter table: params[b][param ...] holds 8 / 32
 *   reals, row-major (re, im) pairs; U2's index is (b_q0 << 1) | b_q1.
 * Further Table 1 gates (2-qubit index (b_q0 << 1) | b_q1):
 *   CY = controlled Y (q0 control), ISWAP = [[1,0,0,0],[0,0,i,0],[0,i,0,0],[0,0,0,1]],
 *   DCX: |x y> -> |y, x xor y> (CNOT q0 -> q1, then CNOT q1 -> q0),
 *   CRZ(t) = diag(1, 1, e^{-it/2}, e^{it/2}), RZZ(t) = exp(-i t Z(x)Z / 2),
 *   CU1(t) = CPHASE(t), RXX(t) / RYY(t) = exp(-i t X(x)X / 2) / exp(-i t Y(x)Y / 2),
 *   RZX(t) = exp(-i t Z(x)X / 2) (Z on q0), ECR = (X(x)I - Y(x)X)/sqrt2,
 *   CH, CSX = controlled H, controlled SX (q0 control);
 *   SX = [[1+i,1-i],[1-i,1+i]]/2, SXDG = SX^dagger;
 *   several angles read from params[b][param ...] (param >= 0 required):
 *   R(t, p) = exp(-i t (cos p X + sin p Y) / 2),
 *   U(t, p, l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]],
 *   CU3(t, p, l) = controlled U, CU(t, p, l, g) = controlled e^{ig} U(t, p, l);
 *   3-qubit monomials, third qubit q2 = sv_gate.index, local index
 *   (b_q0 << 2) | (b_q1 << 1) | b_q2: CCX (Toffoli: q0, q1 controls, q2
 *   target) and CSWAP (Fredkin: q0 control, q1 and q2 exchanged). */
typedef enum sv_gate_kind {
    SV_GATE_I = 0, SV_GATE_X = 1, SV_GATE_Y = 2, SV_GATE_Z = 3, SV_GATE_H = 4,
    SV_GATE_S = 5, SV_GATE_SDG = 6, SV_GATE_T = 7, SV_GATE_TDG = 8,
    SV_GATE_RX = 9, SV_GATE_RY = 10, SV_GATE_RZ = 11, SV_GATE_P = 12,
    SV_GATE_CNOT = 13, SV_GATE_CZ = 14, SV_GATE_SWAP = 15, SV_GATE_CPHASE = 16,
    SV_GATE_MARK = 17, SV_GATE_U1 = 18, SV_GATE_U2 = 19,
    SV_GATE_CY = 20, SV_GATE_ISWAP = 21, SV_GATE_DCX = 22, SV_GATE_CRZ = 23,
    SV_GATE_RZZ = 24, SV_GATE_CU1 = 25, SV_GATE_CCX = 26, SV_GATE_CSWAP = 27,
    SV_GATE_SX = 28, SV_GATE_SXDG = 29, SV_GATE_R = 30, SV_GATE_U = 31,
    SV_GATE_RXX = 32, SV_GATE_RYY = 33, SV_GATE_RZX = 34, SV_GATE_ECR = 35,
    SV_GATE_CH = 36, SV_GATE_CSX = 37, SV_GATE_CU3 = 38, SV_GATE_CU = 39,
    SV_GATE_KIND_COUNT = 40
} sv_gate_kind;

/* One gate, 32 bytes. q1 = -1 for 1-qubit gates and MARK; q0 = -1 for MARK.
 * param = -1: use `angle`; param >= 0: the angle is params[b][param] for batch
 * entry b (see sv_apply_circuit); U1 / U2 require param >= 0 (the first of
 * their 8 / 32 matrix reals), and so do R, U, CU3, CU (the first of their
 * 2 / 3 / 3 / 4 angles). index: basis index of MARK, third qubit of CCX and
 * CSWAP, else ignored. */
typedef struct sv_gate {
    int32_t kind;
    int32_t q0;
    int32_t q1;
    int32_t param;
    double angle;
    uint64_t index;
} sv_gate;

typedef struct sv_state_s *sv_state;

/* Create a batch of `batch` n-qubit states set to |0...0> (Sec. II-A: the
 * register of 2^n amplitudes). 1 <= n_qubits <= 34, batch >= 1.
 * dev_buf: NULL -> the library allocates (hipMalloc) and owns the memory;
 *          else a device buffer of at least batch * 2^n * sizeof(amplitude)
 *          bytes, 256-byte aligned, that the library borrows: the caller keeps
 *          it alive until sv_free returns and the stream work has completed.
 * hip_stream: a hipStream_t or NULL (default stream).
 * |0...0> is recorded, not written: see sv_set_basis.
 * Errors: SV_EINVAL (bad n, dtype, batch, size or alignment), SV_ENOMEM. */
sv_status sv_alloc(int n_qubits, sv_dtype dtype, int batch, void *dev_buf,
                   size_t buf_bytes, void *hip_stream, sv_state *out);

/* Release the handle (and the memory it owns). Waits for its stream. */
sv_status sv_free(sv_state s);

/* Use another HIP stream for the handle's later work. */
sv_status sv_set_stream(sv_state s, void *hip_stream);

/* Set every state of the batch to the basis state |j>, j < 2^n.
 * Like the |0...0> of sv_alloc, the basis state is only recorded here: the
 * first pass of the next sv_apply_circuit generates its amplitudes instead of
 * reading them (Sec. III-B's on-demand idea, with an empty Hadamard mask when
 * no Hadamards lead the circuit), and a readout, sv_sync or sv_device_ptr
 * that comes first writes them. Read the buffer directly only after sv_sync. */
sv_status sv_set_basis(sv_state s, uint64_t j);

/* The caller wrote the amplitudes through the device buffer (for example a
 * borrowed torch tensor): forget any known basis state, so that no Hadamard
 * layer is generated instead of read. */
sv_status sv_mark_modified(sv_state s);

/* Apply the gates in order, in place, to every state of the batch
 * (U_m ... U_1 |psi>, Sec. II-A), asynchronously on the handle's stream.
 * gates: host array of n_gates records, copied before return.
 * params: host array [batch][n_params] (row-major) of angles referenced by
 *         gates with param >= 0, or NULL when no gate references one.
 * Gates are validated first (kind, qubits in range and distinct, MARK index
 * < 2^n, param < n_params); on SV_EINVAL nothing was launched.
 * When the handle is known to hold a basis state |j> (after sv_alloc or
 * sv_set_basis) and the circuit opens with Hadamards, those amplitudes are
 * generated on demand from the RH rule instead of being read (Sec. III-B). */
sv_status sv_apply_circuit(sv_state s, const sv_gate *gates, size_t n_gates,
                           const double *params, size_t n_params);

/* <Z_q> = sum_i |a_i|^2 (1 - 2 b_q(i)) for every batch entry, accumulated in
 * FP64 in a fixed order (Sec. II-A: probabilities are |alpha|^2).
 * out: host array [batch]. Synchronizes the stream. */
sv_status sv_expect_z(sv_state s, int qubit, double *out);

/* sum_i |a_i|^2 per batch entry, FP64 in a fixed order. Sec. II-A: the
 * probabilities |alpha_i|^2 of a valid state sum to 1, so this checks that the
 * gates applied so far kept the state normalized. out: host [batch].
 * Synchronizes the stream. */
sv_status sv_norm(sv_state s, double *out);

/* sv_expect_z / sv_norm without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The same FP64 fixed-order reduction.
 * state: device pointer to `batch` consecutive states of 2^n_qubits amplitudes
 *        of `dtype` (the layout of sv_alloc), 16-byte aligned, on the current
 *        device, read only.
 * qubit: 0..n_qubits-1 for <Z_qubit>, -1 for the norm.
 * out:   device pointer to `batch` doubles, written on hip_stream (a
 *        hipStream_t, or NULL for the default stream); asynchronous, nothing
 *        is synchronized or copied to the host.
 * Partial sums live in a file-scope device array of 65,536 doubles (512 KiB,
 * held on each GPU that runs this call until the process ends):
 * batch * 2^min(max(n_qubits - 12, 0), 10) must not exceed 65,536
 * (so batch <= 64 from n_qubits = 22 up), else SV_EINVAL.
 * Every call on a GPU shares that array: calls that overlap on one GPU (on
 * different streams, or from several host threads) race; serialize them.
 * Errors: SV_EINVAL before anything is launched (NULL or misaligned pointer,
 * dtype, n_qubits outside 1..34, batch outside 1..65535, qubit, scratch
 * size); SV_EDEVICE when the launch fails. */
sv_status sv_expect_z_noalloc(const void *state, int n_qubits, sv_dtype dtype, int batch, int qubit,
                              double *out, void *hip_stream);

/* Amplitudes of batch entry b at k basis indices idx[0..k) (each < 2^n),
 * returned as FP64 (re, im) pairs in out[0 .. 2k). Sec. II-A: the state is
 * the vector of 2^n complex amplitudes alpha_i of the basis states |i>, and
 * |alpha_i|^2 is the probability of measuring i. Complex64 states are widened
 * exactly to FP64. Errors: SV_EINVAL for b outside the batch or an index
 * >= 2^n (nothing launched). Synchronizes the stream. */
sv_status sv_amplitudes(sv_state s, int b, const uint64_t *idx, size_t k, double *out);

/* Adjoint gradient of f_b = <Z_qubit> (of the circuit applied to |0...0>) with
 * respect to params[b][p], for every batch entry b. Runs the forward circuit
 * from |0...0> (the handle ends holding the final states), then one reverse
 * sweep on two states per entry, psi and lambda = Z_qubit psi:
 * for each gate g from last to first, if g is RX/RY/RZ(params[b][p]) then
 * df/dp += Im <lambda|P|psi> (P its Pauli), then psi <- U_g^dagger psi and
 * lambda <- U_g^dagger lambda. Inner products accumulate in FP64.
 * expect: host [batch] (may be NULL); grad: host [batch][n_params], zeroed
 * for parameters no rotation uses. Needs a second device buffer of the
 * handle's size (allocated by the library). Synchronizes the stream.
 * Only RX, RY and RZ may reference parameters (SV_EUNSUPPORTED otherwise). */
sv_status sv_adjoint_expect_z(sv_state s, const sv_gate *gates, size_t n_gates,
                              const double *params, size_t n_params, int qubit,
                              double *expect, double *grad);

/* Wait for the handle's stream; reports asynchronous device faults. */
sv_status sv_sync(sv_state s);

/* Device pointer of batch entry 0 (amplitudes are contiguous). A recorded
 * basis state is written first, asynchronously on the handle's stream. */
void *sv_device_ptr(sv_state s);

/* Tuning and testing options (values are validated, SV_EINVAL otherwise):
 *   SV_OPT_FUSE           1 (default): fuse gates into LDS-tiled passes;
 *                         0: one pass per gate (parity of fused vs unfused).
 *   SV_OPT_MIN_LOW_QUBITS lowest qubits always inside a tile (contiguous HBM
 *                         runs of 2^value amplitudes), 3..7; 0 (default):
 *                         chosen per circuit among 6, 4 and (complex128, still
 *                         128-byte runs) 3 by the planner's cost estimate
 *                         (fewer passes against shorter runs).
 *   SV_OPT_MAX_DENSE      dense gates allowed per pass (ALU budget), >= 1.
 *   SV_OPT_ON_DEMAND_H    1 (default): generate leading Hadamard layers of a
 *                         basis state on demand; 0: apply them as gates.
 *   SV_OPT_SMALL_PATH     1 (default): states of n below the tiled minimum run
 *                         in one workgroup; 2: force that path when n allows.
 *   SV_OPT_PROFILE        1: time every pass kernel with HIP events (see
 *                         sv_profile_read); 0 (default): off.
 *   SV_OPT_REMAP          1 (default): between passes, move the qubits the
 *                         next pass needs onto the contiguous low index bits
 *                         (each pass stores its tile with its own bits
 *                         permuted; the state is back in canonical order
 *                         when sv_apply_circuit's work completes); 0: off.
 *   SV_OPT_PIPELINE       0 (default): one workgroup per tile; 1: passes over
 *                         more tiles than the device holds at once run in a
 *                         persistent kernel whose workgroups load their next
 *                         tile while they apply the pass to the current one
 *                         (LDS exchanges through a half-tile buffer); 2: the
 *                         same with a full-tile buffer. All give the same
 *                         results; 1 and 2 hold two tiles in registers, run at
 *                         fewer waves per SIMD and measured slower on gfx950
 *                         (kept for timing comparisons). */
enum sv_option {
    SV_OPT_FUSE = 1,
    SV_OPT_MIN_LOW_QUBITS = 2,
    SV_OPT_MAX_DENSE = 3,
    SV_OPT_ON_DEMAND_H = 4,
    SV_OPT_SMALL_PATH = 5,
    SV_OPT_PROFILE = 6,
    SV_OPT_REMAP = 7,
    SV_OPT_PIPELINE = 8
};
sv_status sv_set_option(sv_state s, int option, int64_t value);

/* Statistics of the last sv_apply_circuit plan. out[0] = passes,
 * out[1] = register-tile exchanges through LDS, out[2] = gates applied,
 * out[3] = leading Hadamards generated on demand, out[4] = kernel launches,
 * out[5] = algorithmic HBM bytes of the plan (2 * 2^n * amplitude bytes per
 * pass, one read fewer when a pass generates its input), per batch entry,
 * out[6] = permutation gates applied by relabelling the tile addressing,
 * out[7] = leading 1-qubit gates folded into a product state that the first
 * pass generates instead of reading (amp[i] = prod_q u_q[bit q of i]). */
sv_status sv_plan_stats(sv_state s, int64_t out[8]);

/* With SV_OPT_PROFILE on: total milliseconds and count of the pass-kernel
 * launches timed since the last read (HIP events on the handle's stream);
 * resets the counters. Synchronizes the stream. */
sv_status sv_profile_read(sv_state s, double *total_ms, int64_t *launches,
                          double *bytes);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of independent circuit evaluations.
 *
 * A request is an n-qubit circuit applied to |0...0> with its own parameters,
 * answered with <Z_qubit> (FP64). Queued requests are launched in groups:
 *   - small states (n <= 13 for SV_C64, n <= 12 for SV_C128) of any circuit
 *     shape share one launch, one workgroup per request, the state held in
 *     LDS from start to readout (no HBM state at all);
 *   - larger states are grouped with queued requests of the same circuit
 *     (gates and qubit; parameters may differ) and run as one batched set of
 *     fused passes.
 * Up to n_streams groups are in flight on separate HIP streams; whenever one
 * finishes, the oldest queued requests are launched (arrivals do not wait for
 * a batch to drain). A larger-state group is admitted only when its state
 * memory (requests * 2^n * amplitude bytes) fits the engine's HBM budget
 * beside the groups in flight; otherwise it waits. A request's result does
 * not depend on which requests share its launch.
 * The engine is driven by sv_engine_poll; it is not thread-safe. */
typedef struct sv_engine_s *sv_engine;

/* max_batch >= 1: requests per launch group; n_streams in 1..16;
 * hbm_budget_bytes: state memory the engine may hold (0 = no limit). */
sv_status sv_engine_create(sv_dtype dtype, int max_batch, int n_streams,
                           size_t hbm_budget_bytes, sv_engine *out);

/* Stepped engine: continuous batching at pass granularity. Small states are
 * served as above (groups of up to max_small_batch requests on
 * n_small_streams streams). Larger states are admitted, oldest first, while
 * at most max_active of them are on the GPU and their state memory fits the
 * HBM budget; then every step is one launch that runs the next pass of every
 * admitted request, whatever its circuit, n or depth (each on its own state
 * with its own plan), followed by one batched readout of the requests that
 * step completes. Requests that arrive meanwhile join at the next step, so
 * their work overlaps on the device with the requests already running. A
 * request's first pass generates its initial product state (its leading
 * 1-qubit gates applied to |0...0>, on demand) instead of reading a filled
 * state. Every request runs the same code whatever shares its steps, so its
 * result does not depend on the mix. A finished request's state buffer is
 * kept for the next request of the same n; kept buffers count against a
 * nonzero HBM budget and are given back when a request needs new memory,
 * and with no budget (0) they stay with the engine until sv_engine_free.
 * The plan arena holds 256 MiB of op records (requests wait when it is
 * full) and 32 MiB of distinct circuits (SV_ENOMEM beyond). */
sv_status sv_engine_create_stepped(sv_dtype dtype, int max_active, int max_small_batch, int n_small_streams,
                                   size_t hbm_budget_bytes, sv_engine *out);

/* Waits for the groups in flight, then frees the engine. */
sv_status sv_engine_free(sv_engine e);

/* Queue one request (gates and params are copied). n_params reals of
 * parameters (may be 0 with params NULL); qubit: the measured qubit.
 * Gates are validated as in sv_apply_circuit (SV_EINVAL, nothing queued);
 * n_qubits above 30 is SV_EUNSUPPORTED; a state larger than a nonzero HBM
 * budget is SV_ENOMEM (it could never be admitted). */
sv_status sv_engine_submit(sv_engine e, uint64_t id, int n_qubits, const sv_gate *gates,
                           size_t n_gates, const double *params, size_t n_params, int qubit);

/* Register a circuit with the engine once (validated and planned now, as
 * in sv_engine_submit) for repeated submissions with other parameters:
 * *circuit receives its handle (the same handle for the same circuit). */
sv_status sv_engine_register(sv_engine e, int n_qubits, const sv_gate *gates, size_t n_gates, size_t n_params,
                             int qubit, int64_t *circuit);

/* Queue one evaluation of a registered circuit with its own parameters
 * (exactly the registered n_params reals, copied). SV_EINVAL for a handle
 * this engine did not return, another parameter count, or NULL params with
 * n_params > 0; nothing is queued then. */
sv_status sv_engine_submit_registered(sv_engine e, uint64_t id, int64_t circuit, const double *params,
                                      size_t n_params);

/* Retire finished groups, launch queued requests as streams and memory
 * allow, and return up to `cap` finished results (ids[i], values[i]) in
 * *count. wait_us > 0: wait up to that many microseconds for at least one
 * result. */
sv_status sv_engine_poll(sv_engine e, int64_t wait_us, uint64_t *ids, double *values,
                         size_t cap, size_t *count);

/* out[0] queued, out[1] in flight (requests), out[2] completed,
 * out[3] groups launched, out[4] state bytes held, out[5] largest group,
 * out[6] groups refused for memory (deferred), out[7] small-state groups. */
sv_status sv_engine_stats(sv_engine e, int64_t out[8]);

/* Description of the last error on this thread ("" if none). */
const char *sv_last_error(void);

/* Library version string. */
const char *sv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
