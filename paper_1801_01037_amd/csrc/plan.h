// Circuit planning: fusion of gate runs into passes, and their execution.
#pragma once

#include <string>

#include "sv_internal.h"

namespace svk {

// Plans and queues a validated gate list with SV_FUSE / SV_FUSE_DENSE /
// SV_GRAPH. On failure returns a status and sets *err.
sv_status plan_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                   std::string *err);

// Queues a general gate U (2^k x 2^k complex, row major, FP64) on the k
// validated, distinct qubits q[0..k-1], 2 <= k <= 5: as one dense 5-qubit
// block on the matrix cores when n >= 9 (U padded with the identity on the
// highest unused qubits), else with the small-register kernel.
sv_status apply_unitary(sv_state s, const int32_t *q, int k, const double *u, std::string *err);

// Frees planning buffers and cached graphs owned by the handle.
void plan_release(sv_state s);

// Plans without a device: gate_op[i] (n_gates entries, may be NULL) receives
// the index, in execution order, of the last op that carries gate i.
// Plans a validated gate list into tile passes (K = 4 geometry) and uploads
// them; the plan object is owned by the caller (sv_plan_destroy).
sv_status plan_create(sv_state s, const sv_gate *gates, size_t n_gates, sv_plan *out,
                      std::string *err);

int plan_dense_inspect(int n, const sv_gate *gates, size_t n_gates, uint64_t *masks,
                       double *mats, int cap);
int plan_inspect(int n, sv_dtype dt, const sv_gate *gates, size_t n_gates, bool relabel,
                 int32_t *gate_op,
                 int32_t *n_passes, int32_t *n_groups, int32_t *n_ops);

}  // namespace svk
