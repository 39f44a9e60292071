// Gate classification and pass planning (host side).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <memory>
#include <vector>

#include "../../include/sv.h"
#include "sv_plan.hpp"

namespace sv {

// Gate classes (the gate-local compressed forms):
//   D1/D2   diagonal: 2 or 4 phases (one non-zero per row, on the diagonal)
//   MARK    n-qubit diagonal with a single -1 (value + index)
//   X/Y/CX/SWAP  monomial: one non-zero per row, a permutation with phases
//                (the DAX entry restricted to the gate's own 2^k x 2^k matrix)
//   H       a Hadamard: one magnitude and on-demand signs (RH)
//   DENSE1  general 2x2
//   DENSE2  general 4x4 (matrix gate U2)
enum GClass : uint8_t {
    G_NOP = 0, G_D1, G_D2, G_MARK, G_X, G_Y, G_CX, G_SWAP, G_H, G_DENSE1, G_DENSE2, G_CCX
};

struct CGate {
    GClass cls = G_NOP;
    int q0 = -1, q1 = -1;   // 2-qubit: q0 is the high local bit (CX: control)
    int q2 = -1;            // CCX: target (q0, q1 controls)
    int src = -1;           // index in the caller's gate list
    uint64_t index = 0;     // MARK basis index
    uint64_t support = 0;   // qubit mask the gate acts on
    uint64_t qneed = 0;     // qubits that must be tile qubits of its pass
    uint64_t rneed = 0;     // qubits that must sit in register bits when applied
    bool diag = false;
};

// Small-path constant block: `count` reals per batch entry at offset `off`.
enum ConstKind : uint8_t { CK_D1 = 1, CK_D2, CK_DENSE1, CK_HMAT, CK_DENSE2 };
struct ConstBlock {
    ConstKind kind;
    int gate;
    uint64_t off;
};

// A 2x2 factor of a composed register-bit operation; conj_x: the factor acts
// on a label whose XOR bit is set, so its physical matrix is X G X.
enum FactorKind : uint8_t { FK_GATE = 0, FK_X, FK_YDIAG, FK_H };
struct Factor {
    uint8_t kind;
    bool conj_x;
    int gate;
};

enum PayloadKind : uint8_t {
    PK_NONE = 0,
    PK_MAT2,    // the 2x2 product of `factors`
    PK_MAT2RI,  // the real R of that product written as diag(i^g0, i^g1) R diag(1, i^bt)
                // (g0, g1, bt: bits 0..2 of hdr.b)
    PK_DIAG2,   // its two diagonal entries
    PK_D4,      // the 2-qubit diagonal gate's entries, permuted by perm
    PK_SCALE,   // one real
    PK_SIDE,    // one diagonal entry of the product of `factors` (hdr.b: 0 or 1)
    PK_G3,      // entry 3 of the 2-qubit diagonal gate (its one non-trivial entry)
    PK_UDN,     // C and the term ratios of the merged uniform diagonals `ucon`
    PK_MAT4,    // a U2 gate's 4x4 matrix, rows and columns permuted by perm (16 entries,
                // continued in the records that follow the operation)
    PK_CONT,    // continuation record of the preceding PK_MAT4 (entries from `gate` e0)
    PK_PROD,    // product-state vectors u_q = M_q e_(bit q of basis) of the qubits
                // qfirst .. qfirst + per - 1, M_q the product of qgates[q] in order
};

// One diagonal gate on thread or tile-base bits inside a merged OP_UDN.
// With P(x, y) its value at source bits (x, y) (1-qubit gates: y = 0),
// C *= P(0, 0) and the ratios P(1,0)/P(0,0) (term t0), P(0,1)/P(0,0) (t1)
// and P(1,1) P(0,0) / (P(1,0) P(0,1)) (t01) multiply their terms.
enum UContribKind : uint8_t { UC_D1 = 1, UC_D2, UC_YDIAG };
struct UContrib {
    int gate = -1;
    uint8_t kind = UC_D1;
    bool inv = false;                // 1-qubit: the label's XOR bit (values swapped)
    uint8_t perm[4] = {0, 1, 2, 3};  // 2-qubit: (x << 1) | y -> gate-local index
    int8_t t0 = -1, t1 = -1, t01 = -1;
};

// A pass operation plus the recipe of its payload (materialized per batch
// entry from the gates' angles).
struct HostOp {
    DevOp hdr{};
    uint8_t pk = PK_NONE;
    std::vector<Factor> factors;   // PK_MAT2 / PK_DIAG2 / PK_SIDE: product, first factor applied first
    int gate = -1;                 // PK_D4 / PK_G3: the 2-qubit diagonal gate
    uint8_t perm[4] = {0, 1, 2, 3};  // PK_D4: payload entry e takes the gate's diagonal entry perm[e]
    std::vector<UContrib> ucon;    // PK_UDN
    int n_terms = 0;               // PK_UDN
    double scale = 1.0;
    int qfirst = 0;                // PK_PROD
    int qcount = 0;
    uint64_t basis = 0;
    std::shared_ptr<const std::vector<std::vector<int>>> qgates;   // PK_PROD: caller gate
                                                                   // indices per qubit
};

struct PlanOptions;
bool same_options(const PlanOptions &a, const PlanOptions &b);

struct PlanOptions {
    int R = 4;            // register bits per thread
    int v = 0;            // vector bits (complex64: 1, label 0 in register 0 for 16-byte I/O)
    int m = 3;            // swizzle width (3 for 16-byte slots, 4 for 8-byte)
    int c = 6;            // lowest qubits always in the tile
    bool auto_low = false;  // build_plan_auto: choose c among 6, 4 and (complex128) 3
    int w_max = 8;        // thread bits of a full workgroup
    bool fuse = true;     // false: one pass per gate
    bool remap = true;    // permute the tile's address bits at each store (see build_plan)
    int max_dense = 1 << 20;  // dense register operations (DENSE1) per pass
    bool gen_h = true;    // generate leading Hadamards of a basis state
    bool basis_known = false;
    uint64_t basis_j = 0;
    bool gen_basis = false;   // the memory does not hold that basis state yet: the
                              // first pass generates it (an empty Hadamard mask
                              // when no Hadamards lead the circuit)
    int ud_max = 3;       // terms of a merged uniform-diagonal operation
    int small_max = 12;   // largest n of the one-workgroup path
    int small_mode = 1;   // 1: use it below the tiled minimum; 2: whenever n allows
};

struct Plan {
    bool small = false;
    int n = 0;
    std::vector<DevPass> passes;
    std::vector<DevLayout> layouts;
    std::vector<HostOp> ops;
    std::vector<SmallOp> sops;
    std::vector<ConstBlock> cblocks;   // small path
    uint64_t cstride = 0;              // small path: reals per batch entry
    int64_t n_exch = 0;
    int64_t n_gen_h = 0;
    int64_t n_gen_product = 0;         // leading 1-qubit gates folded into a generated product state
    int64_t gates_applied = 0;
    int64_t n_relabel = 0;             // permutation gates absorbed into layouts
    int64_t n_restore = 0;             // passes that only put qubits back on their own bits
    int low = 0;                       // contiguous low qubits of every tile (c)
};

// Structural classification of a validated gate (independent of the angle).
CGate classify(const sv_gate &g, int n, int src);

// Validate gates; on error returns false and fills `err`.
bool validate_gates(int n, const sv_gate *gates, size_t n_gates, size_t n_params,
                    bool params_given, std::string &err);

// Build the plan. Gates must be validated.
Plan build_plan(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt);
// With opt.auto_low, the plan of lower estimated cost among c = 6 and c = 4
// contiguous low qubits (fewer, fuller passes against shorter contiguous HBM
// runs); otherwise build_plan.
Plan build_plan_auto(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt);

// Tiled path: write [batch][ops.size()] DevOp records with their payloads.
void materialize_ops(const Plan &p, const sv_gate *gates, const double *params,
                     size_t n_params, int batch, bool f32, void *out);

// Small path: fill the constant table [batch][cstride] (double or float).
void materialize_consts(const Plan &p, const sv_gate *gates, const double *params,
                        size_t n_params, int batch, bool f32, void *out);

// Tiled-path geometry for n qubits: k (tile qubits) and w (thread bits), or
// false when n is too small for a full wave of the tiled kernel.
bool tile_geometry(int n, const PlanOptions &opt, int &k, int &w);

}  // namespace sv
