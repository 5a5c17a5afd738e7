// Circuit planning: fusion of gate runs into passes, and their execution.
#pragma once

#include <string>
#include <vector>

#include "dense.h"
#include "tile.h"

#include "sv_internal.h"

namespace svk {

// Plans and queues a validated gate list with SV_FUSE / SV_FUSE_DENSE (SV_GRAPH
// is handled by circuit_graph_run). On failure returns a status and sets *err.
sv_status plan_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                   std::string *err);

// Queues a general gate U (2^k x 2^k complex, row major, FP64) on the k
// validated, distinct qubits q[0..k-1], 2 <= k <= 5: as one dense 5-qubit
// block on the matrix cores when n >= 9 (U padded with the identity on the
// highest unused qubits), else with the small-register kernel.
sv_status apply_unitary(sv_state s, const int32_t *q, int k, const double *u, std::string *err);

// Frees planning buffers and cached graphs owned by the handle.
void plan_release(sv_state s);

// Plans a validated gate list into tile passes (K = 4 geometry) and uploads
// them; the plan object is owned by the caller (sv_plan_destroy).
// relabel = false keeps the standard storage order between passes
// (SV_NO_RELABEL).
sv_status plan_create(sv_state s, const sv_gate *gates, size_t n_gates, sv_plan *out,
                      std::string *err, bool relabel = true);

// The tile passes SV_FUSE makes of a validated gate list (any n), their tables
// uploaded once (synchronously) to a device buffer *dev that the caller frees;
// *launches receives the arguments of one launch_tile per pass, in order, all
// with register bits *K.
struct JitKernel;
// jit: if not null, also compiles the passes (SV_JIT) into (*jit)[p].
sv_status tiles_prepare(sv_state s, const sv_gate *gates, size_t n_gates, bool relabel, void **dev,
                        std::vector<TileArgs> *launches, int *K, std::vector<JitKernel> *jit,
                        std::string *err);

// The dense 5-qubit blocks of a validated gate list (n >= 9), their matrices
// uploaded once (synchronously) to a device buffer *dev that the caller frees;
// *launches receives one launch per block, in order.
sv_status dense_prepare(sv_state s, const sv_gate *gates, size_t n_gates, void **dev,
                        std::vector<DenseArgs> *launches, std::string *err);

// SV_GRAPH for one circuit on one state (flags: SV_GRAPH with 0, SV_FUSE,
// SV_FUSE | SV_NO_RELABEL or SV_FUSE_DENSE): the launches are captured in a
// HIP graph the first time a gate list is run on the handle and replayed while
// the same list comes back. Validated gates only.
sv_status circuit_graph_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                            std::string *err);
// Frees the handle's captured circuit graph and the buffers it reads.
void circuit_graph_release(sv_state s);

// A tile pass compiled for its own program (jit.hip).
struct JitKernel {
    hipFunction_t fn;   // null: the pass runs with the generic tile kernel
    int per_cu;         // resident work-groups per CU
};
// Compiles (or finds in the process's cache) one kernel per pass of a plan;
// groups and ops are the plan's host records (TileArgs.group0 and the groups'
// op0 index them). On failure returns SV_EDEVICE with the compiler's log.
sv_status jit_passes(sv_dtype dt, int K, const std::vector<TileArgs> &passes,
                     const std::vector<TileGroup> &groups, const std::vector<TileOp> &ops,
                     std::vector<JitKernel> *out, std::string *err);
// Compiles the distinct programs of a plan's passes on the host only (no
// device is touched, nothing is cached); *n_programs receives their number.
bool jit_compile_only(sv_dtype dt, int K, const std::vector<TileArgs> &passes,
                      const std::vector<TileGroup> &groups, const std::vector<TileOp> &ops,
                      int32_t *n_programs, std::string *err);
// Host-only: plans a validated gate list as SV_FUSE does and compiles its pass
// programs (jit_compile_only). 0 on success, -1 planning failed, -2 compiling.
int plan_jit_check(int n, sv_dtype dt, const sv_gate *gates, size_t n_gates, bool relabel,
                   int32_t *n_programs, std::string *err);
// Launches pass `a` (its device pointers patched) with its compiled kernel,
// or with the generic one when it has none.
hipError_t jit_launch(const JitKernel &k, const TileArgs &a, int K, bool c64, hipStream_t st);

// One gate as its own launch (sv_api.hip).
sv_status queue_gate(sv_state s, const sv_gate &g);

int plan_dense_inspect(int n, const sv_gate *gates, size_t n_gates, uint64_t *masks,
                       double *mats, int cap);
// Plans without a device: gate_op[i] (n_gates entries, may be NULL) receives
// the index, in execution order, of the last op that carries gate i.
int plan_inspect(int n, sv_dtype dt, const sv_gate *gates, size_t n_gates, bool relabel,
                 int32_t *gate_op,
                 int32_t *n_passes, int32_t *n_groups, int32_t *n_ops);

}  // namespace svk
