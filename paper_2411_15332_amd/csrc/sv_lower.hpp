// Host lowering of composite Table 1 gates into the planner's kinds.
//
// Each rule is an exact identity between operators (phases i and -1 are
// exact; derived angles are one FP64 multiplication):
//   CY(c, t)        = S_t CNOT(c, t) SDG_t
//   ISWAP(a, b)     = SWAP(a, b) S_a S_b CZ(a, b)          (diag(1, i, i, 1), then SWAP)
//   DCX(a, b)       = CNOT(b, a) CNOT(a, b)
//   CRZ(c, t; x)    = CPHASE(c, t; x) P_c(-x/2)
//   RZZ(a, b; x)    = CPHASE(a, b; -2x) P_b(x) RZ_a(x)
//   CU1(a, b; x)    = CPHASE(a, b; x)
//   CSWAP(c; a, b)  = CNOT(b, a) CCX(c, a -> b) CNOT(b, a)
//   SX = H S H, SXDG = H SDG H
//   R(t, p)         = RZ(p) RX(t) RZ(-p)
//   U(t, p, l)      = P(p) RY(t) P(l)
//   RXX(x)          = (H (x) H) RZZ(x) (H (x) H)
//   RYY(x)          = (S (x) S) RXX(x) (SDG (x) SDG)
//   RZX(x)          = (I (x) H) RZZ(x) (I (x) H)
//   ECR             = RZX(-pi/4) X_a RZX(pi/4)
//   CH(c, t)        = RY_t(pi/4) CZ RY_t(-pi/4)
//   CSX(c, t)       = H_t CPHASE(pi/2) H_t
//   CU3(t, p, l)    = CPHASE(p) CRY(t) CPHASE(l), CRY(t) = CNOT RY(-t/2) CNOT RY(t/2)
//   CU(t, p, l, g)  = P_c(g) CU3(t, p, l)
// (operators written right to left: the rightmost is applied first). CCX is
// not lowered: it is a monomial the pass kernel applies directly.
#pragma once

#include <cstddef>
#include <vector>

#include "../../include/sv.h"

namespace sv {

struct Lowering {
    std::vector<sv_gate> gates;   // planner kinds only (kind < SV_GATE_CY, or CCX)
    // Derived parameter column n_params + i holds params[src[i]] * scale[i].
    std::vector<int> src;
    std::vector<double> scale;
    bool changed = false;         // some gate was rewritten
};

// Lower `n` validated gate records; parameters of lowered parametric gates
// that need a multiple of the caller's angle get derived columns.
void lower_gates(const sv_gate *g, size_t n, size_t n_params, Lowering &out);

// The caller's [batch][n_params] table extended by the derived columns:
// [batch][n_params + src.size()]. Empty when no column is derived.
void lower_params(const Lowering &L, const double *params, size_t n_params, int batch,
                  std::vector<double> &out);

}  // namespace sv
