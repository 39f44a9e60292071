// Gate classification and pass planning (host side).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
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
//   DENSE1/DENSE2  general 2x2 / 4x4
enum GClass : uint8_t {
    G_NOP = 0, G_D1, G_D2, G_MARK, G_X, G_Y, G_CX, G_SWAP, G_H, G_DENSE1, G_DENSE2
};

struct CGate {
    GClass cls;
    int q0 = -1, q1 = -1;   // 2-qubit: q0 is the high local bit (CX: control)
    int src = -1;           // index in the caller's gate list
    uint64_t index = 0;     // MARK basis index
    uint64_t support = 0;   // qubit mask the gate acts on
    uint64_t need = 0;      // qubits that must be register bits to apply it
    bool diag = false;
};

// Constant block of one op: `count` reals per batch entry at offset `off`.
enum ConstKind : uint8_t { CK_D1 = 1, CK_D2, CK_DENSE1, CK_DENSE2, CK_SCALE, CK_HMAT };
struct ConstBlock {
    ConstKind kind;
    int gate;          // source gate index (for its kind / angle)
    double scale;      // real factor folded into the block (Hadamard magnitude)
    uint64_t off;      // offset in reals within a batch entry
    bool swap_bits;    // DENSE2 / D2 stored with its two local bits exchanged
};

struct PlanOptions {
    int R = 4;            // register bits per thread
    int v = 0;            // vector bits (complex64: 1, local bit 0 in register 0)
    int m = 3;            // swizzle width (3 for 16-byte slots, 4 for 8-byte)
    int c = 6;            // lowest qubits always in the tile
    int w_max = 8;        // thread bits of a full workgroup
    bool fuse = true;     // false: one pass per gate
    int max_dense = 1 << 20;  // dense ops (DENSE1/DENSE2) per pass
    bool gen_h = true;    // generate leading Hadamards of a basis state
    bool basis_known = false;
    uint64_t basis_j = 0;
    int small_max = 12;   // largest n of the one-workgroup path
    int small_mode = 1;   // 1: use it below the tiled minimum; 2: whenever n allows
};

struct Plan {
    bool small = false;
    int n = 0;
    std::vector<DevPass> passes;
    std::vector<DevLayout> layouts;
    std::vector<DevOp> ops;
    std::vector<SmallOp> sops;
    std::vector<ConstBlock> cblocks;
    uint64_t cstride = 0;     // reals per batch entry
    int64_t n_exch = 0;
    int64_t n_gen_h = 0;
    int64_t gates_applied = 0;
};

// Structural classification of a validated gate (independent of the angle).
CGate classify(const sv_gate &g, int n, int src);

// Validate gates; on error returns false and fills `err`.
bool validate_gates(int n, const sv_gate *gates, size_t n_gates, size_t n_params,
                    bool params_given, std::string &err);

// Build the plan. Gates must be validated.
Plan build_plan(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt);

// Fill the constant table [batch][cstride] (double or float).
void materialize_consts(const Plan &p, const sv_gate *gates, const double *params,
                        size_t n_params, int batch, bool f32, void *out);

// Tiled-path geometry for n qubits: k (tile qubits) and w (thread bits), or
// false when n is too small for a full wave of the tiled kernel.
bool tile_geometry(int n, const PlanOptions &opt, int &k, int &w);

}  // namespace sv
