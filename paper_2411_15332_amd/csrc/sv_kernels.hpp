// Host-side launchers of the gfx950 kernels (defined in sv_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sv_plan.hpp"

namespace sv {

// Tile geometry of the pass kernel, per precision: 2^R amplitudes in the
// registers of each of 2^W threads, a tile of 2^(R+W) amplitudes, exchanged
// through a half-tile LDS buffer.
//   complex128: R = 4, W = 8: 4096 amplitudes, 32 KiB of LDS per workgroup
//   complex64:  R = 5, W = 8: 8192 amplitudes, 32 KiB of LDS per workgroup
// (512-thread workgroups with 8192-amplitude complex128 tiles save passes but
// ran each pass about twice as long on gfx950. Complex128 with R = 5, W = 7
// saves exchanges but needs 174 VGPRs: measured 3% slower on a depth-100
// random circuit and 16% slower on latency-bound Grover passes.)
constexpr int kRegBitsC128 = 4;
constexpr int kThreadBitsC128 = 8;
constexpr int kRegBitsC64 = 5;
constexpr int kThreadBitsC64 = 8;
constexpr int kMinThreadBits = 6;    // at least one full 64-lane wave
static_assert(kThreadBitsC128 <= kLayoutThreadBits && kThreadBitsC64 <= kLayoutThreadBits, "");
static_assert(kRegBitsC128 <= kLayoutRegBits && kRegBitsC64 <= kLayoutRegBits, "");

// Largest state (qubits) the one-workgroup kernel keeps in 64 KiB of LDS.
constexpr int kSmallMaxQubitsC128 = 12;
constexpr int kSmallMaxQubitsC64 = 13;

// dt: 1 = complex64, 2 = complex128 (the sv_dtype values).
hipError_t launch_fill_basis(int dt, void *state, uint64_t n_amps, int batch,
                             uint64_t j, hipStream_t st);

// One pass over `batch` states. pipeline 1 (2): passes of more tiles than
// fit on the device at once run in the persistent kernel that loads each
// workgroup's next tile during the current one's operations, exchanging
// through a half-tile (full-tile) LDS buffer; 0: one workgroup per tile.
// Passes with a 4x4 gate and small launches always run one workgroup per tile.
hipError_t launch_pass(int dt, void *state, uint64_t n_amps, int batch,
                       const DevPass *d_passes, int pass_idx, const DevPass &h_pass,
                       const DevLayout *d_layouts, const DevOp *d_ops, uint64_t ops_stride,
                       int pipeline, hipStream_t st);

hipError_t launch_small(int dt, void *state, int n, int batch, const SmallOp *d_ops,
                        int n_ops, const void *d_consts, uint64_t const_stride,
                        hipStream_t st);

// Continuous batching: one launch runs the current pass of several requests,
// each on its own state with its own plan (records at byte offsets in
// d_arena; items: one workgroup per tile; every pass of the launch generates
// its input (gen) or none does, and holds a 4x4 gate (d2) or none does).
hipError_t launch_pass_multi(int dt, const void *d_arena, const StepReq *d_reqs, const StepItem *d_items,
                             uint32_t n_items, bool gen, bool d2, hipStream_t st);
// Readouts of several states: items are (state, block) pieces of the
// single-state reduction (reduce_blocks(n) blocks of reduce_chunk(n)
// amplitudes each), summed in the same order; fin items give each result's
// range of partials and its slot in d_out.
int reduce_blocks(int n);
size_t reduce_chunk(int n);
hipError_t launch_reduce_multi(int dt, const RedItem *d_items, uint32_t n_items, double *d_part,
                               const FinItem *d_fin, uint32_t n_fin, double *d_out, hipStream_t st);

// Per-state sum of |a_i|^2 * (qubit < 0 ? 1 : 1 - 2 b_qubit(i)) in FP64.
// d_partials needs reduce_partials_size(n) * batch doubles; d_out batch doubles.
size_t reduce_partials_size(int n);
// partial sums per (batch entry, term) of the adjoint inner products
size_t pauli_ip_partials_size(int n);
hipError_t launch_reduce(int dt, const void *state, int n, int batch, int qubit,
                         double *d_partials, double *d_out, hipStream_t st);

// Capacity (doubles) of the file-scope partial-sum array of the
// allocation-free readout, and its device address on the current device
// (looked up once per device).
constexpr size_t kStaticPartials = size_t(1) << 16;
hipError_t static_partials(double **out);

// out[2i], out[2i+1] = FP64 (re, im) of amplitude idx[i] of the state at `state`.
hipError_t launch_gather(int dt, const void *state, const uint64_t *d_idx, size_t k,
                         double *d_out, hipStream_t st);

// lambda = Z_q psi for `batch` consecutive states.
hipError_t launch_copy_z(int dt, const void *psi, void *lam, uint64_t n_amps, int batch, int q,
                         hipStream_t st);

// Adjoint inner products Im <lambda_b | P | psi_b>, P = X (1), Y (2) or Z (3)
// on one qubit, accumulated in FP64 in a fixed order. Several (qubit, Pauli)
// terms of one adjoint run go by value in one launch.
constexpr int kMaxIpTerms = 32;
constexpr int kIpMaxXYTerms = 12;   // X / Y terms of one contiguous-chunk launch (qubits < 12)
struct IpTerms {
    uint8_t q[kMaxIpTerms];
    uint8_t pauli[kMaxIpTerms];   // 1 = X, 2 = Y, 3 = Z
};
struct IpOffsets {
    uint64_t off[kMaxIpTerms];    // gradient index of each term within a batch row
};
// grad[b * grad_stride + off[t]] += Im <lambda_b | P_t | psi_b> for nt <= kMaxIpTerms
// terms in one read of the states. Z terms take any qubit; X and Y terms need
// qubit < pauli_ip_multi_chunk_bits(n) (hipErrorInvalidValue otherwise).
// d_partials holds batch * nt * pauli_ip_partials_size(n) doubles.
hipError_t launch_pauli_ip_multi(int dt, const void *psi, const void *lam, int n, int batch,
                                 const IpTerms &terms, const IpOffsets &offs, int nt, double *d_partials,
                                 double *d_grad, uint64_t grad_stride, hipStream_t st);
int pauli_ip_multi_chunk_bits(int n);

// The same for up to kMaxIpHiTerms X and Y terms on qubits at or above bit
// 12: the sub-chunks staged in LDS are the 2^12 amplitudes spanned by qubits
// 0 .. 11 - h and the h <= 8 qubits hq[] (ascending). A term's q is its
// qubit's position in that set (q < 12 - h for a low qubit, 12 - h + k for
// hq[k]). Needs n >= 13 (hipErrorInvalidValue otherwise).
constexpr int kMaxIpHiTerms = 8;
struct IpHiMap {
    uint8_t hq[8];
    int32_t h;
};
hipError_t launch_pauli_ip_hi(int dt, const void *psi, const void *lam, int n, int batch,
                              const IpTerms &terms, const IpOffsets &offs, int nt, const IpHiMap &map,
                              double *d_partials, double *d_grad, uint64_t grad_stride, hipStream_t st);

// One workgroup per job: |0...0> in LDS, the job's small ops, out[j] = <Z_qubit>.
hipError_t launch_small_jobs(int dt, const SmallJob *d_jobs, int n_jobs, const SmallOp *d_ops,
                             const void *d_consts, double *d_out, hipStream_t st);

}  // namespace sv
