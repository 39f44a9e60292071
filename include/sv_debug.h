/*
 * sv_debug.h — diagnostics of the state-vector library (no device work).
 */
#ifndef SV_DEBUG_H
#define SV_DEBUG_H

#include <stddef.h>
#include <stdint.h>

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Build the pass plan that sv_apply_circuit would run for `gates` on an n-qubit
 * state of `dtype`, without touching a GPU, and serialize it into `out`.
 * opts (may be NULL for defaults): [0] fuse (0/1), [1] lowest qubits kept in a
 * tile (3..7, or 0 for the planner's choice), [2] dense gates per pass, [3] on-demand Hadamards (0/1),
 * [4] state is a known basis state (0/1), [5] that basis index, [6] small-path
 * mode (1 or 2), [7] qubit remapping (0/1) — the meanings of the matching
 * SV_OPT_* options — and [8] the basis state of [4]/[5] is only recorded, not
 * yet written to memory (0/1: the first pass generates it, as after sv_alloc
 * or sv_set_basis). opts, when given, holds these 9 values.
 * Layout of `out`: 256-byte header of int64 fields
 *   [0] small path, [1] passes, [2] layouts, [3] ops, [4] small ops,
 *   [5] constant reals per batch entry, [6] exchanges, [7] generated
 *   Hadamards, [8] gates applied, [9] k, [10] w, [11] R, [12] swizzle width,
 *   [13..17] byte offsets of the pass, layout, op, small-op and constant
 *   arrays, [18] algorithmic HBM bytes, [19] relabelled permutation gates,
 *   [20] passes that only put qubits back on their own bits, [21] contiguous
 *   low qubits of every tile (opts[1], or the planner's choice when it is 0),
 *   [22] leading 1-qubit gates folded into the generated product state,
 * followed by those arrays (constants in the state's precision: FP64 for
 * SV_C128, FP32 for SV_C64; batch entry 0).
 * Returns the number of bytes the dump needs (nothing is written when `out`
 * is NULL or `cap` is smaller), or a negative sv_status on bad input. */
int64_t sv_debug_plan(int n, int dtype, const sv_gate *gates, size_t n_gates,
                      const double *params, size_t n_params, const int64_t *opts,
                      void *out, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* SV_DEBUG_H */
