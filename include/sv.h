/*
 * sv.h -- C ABI of the MI355X state-vector simulator (libsv.so).
 *
 * The problem it solves is the one stated in R. LaRose, "Distributed Memory
 * Techniques for Classical Simulation of Quantum Circuits" (arXiv:1801.01037),
 * section State Vector Partitioning:
 *   - an n-qubit register is the vector of 2^n complex amplitudes
 *     alpha_{b_{n-1}...b_0}, indexed in binary (the three-qubit
 *     binary-index equation);
 *   - a one-qubit gate Q = [[q11, q12], [q21, q22]] on qubit i replaces every
 *     pair of amplitudes whose indices differ only in bit i by
 *     (q11 a + q12 b, q21 a + q22 b) (the stride update equation);
 *   - a gate with control c and target t does the same only where bit c of
 *     the index is one (caption of Algorithm 1);
 *   - a circuit is a sequence of such gates (Quantum Circuits).
 *
 * Conventions shared by every entry point:
 *   - Qubit q is bit q of the amplitude index (stride 2^q). Valid n: 1..34.
 *   - Amplitudes are stored contiguously and interleaved (re, im): float2 for
 *     SV_C64 (8 bytes each), double2 for SV_C128 (16 bytes each); the layout of
 *     torch.complex64 / torch.complex128.
 *   - Gate matrices are always passed as 8 doubles: q11, q12, q21, q22 as
 *     (re, im) pairs, row major. They are read during the call only. For
 *     SV_C64 they are rounded once to float. Unitarity is assumed, not checked.
 *   - Asynchrony: calls that change the state enqueue work on the handle's
 *     HIP stream and return. Device faults surface as SV_EDEVICE from the next
 *     call that synchronises (sv_probs, sv_norm, sv_copy_out, sv_synchronize).
 *   - Errors: every call returns an sv_status; SV_OK is 0. The message of the
 *     last failure on the calling thread is in sv_last_error(). No C++
 *     exception crosses this boundary. A failed call leaves the state as it
 *     was unless the status is SV_EDEVICE.
 *   - Threads: one handle must not be used from two threads at once; distinct
 *     handles may be used concurrently.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_state_s *sv_state;   /* opaque handle */

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

typedef enum {
    SV_OK = 0,
    SV_EINVAL = -1,        /* bad argument: null pointer, qubit out of range, ... */
    SV_ENOMEM = -2,        /* device or host allocation failed */
    SV_EDEVICE = -3,       /* a HIP runtime call or a kernel failed */
    SV_EUNSUPPORTED = -4   /* valid request this build does not serve */
} sv_status;

/* Gate kinds of sv_gate.kind. */
enum {
    SV_G_U = 0,       /* 2x2 matrix m on `target`; `control` must be -1            */
    SV_G_CU = 1,      /* 2x2 matrix m on `target` where bit `control` is 1 (CNOT:  */
                      /* m = X)                                                    */
    SV_G_CPHASE = 2,  /* diag(1, e^{i theta}) on `target` where bit `control` is 1; */
                      /* theta = m[0] in radians (controlled-phase R_k has         */
                      /* theta = 2 pi / 2^k)                                       */
    SV_G_MCU = 3,     /* 2x2 matrix m on `target` where every bit of a control     */
                      /* mask is 1 (Toffoli: two controls, m = X); the mask's low  */
                      /* 32 bits are in `control`, its high 32 bits in `flags`    */
    SV_G_UNITARY = 4  /* a general gate on k = `control` qubits (1 <= k <= 5), as  */
                      /* sv_apply_unitary applies it: qubit j of its list in bits  */
                      /* 6j..6j+5 of `flags` (j = 0 is the least significant bit  */
                      /* of the local index); `target` = index of its matrix in    */
                      /* the table given to sv_run_circuit_ex; m unused           */
};

/* One gate of a circuit: 80 bytes, the same record the seeded generators
 * write. `flags` must be 0 except for SV_G_MCU and SV_G_UNITARY. */
typedef struct {
    int32_t kind;
    int32_t control;    /* -1 when the gate has no control */
    int32_t target;
    int32_t flags;
    double m[8];        /* q11, q12, q21, q22 as (re, im); SV_G_CPHASE: m[0] = theta */
} sv_gate;

/* sv_run_circuit flags. With no flag every gate is its own kernel launch
 * (one pass over the state per gate). */
#define SV_FUSE        1u  /* group gates into LDS-tile passes: each pass reads and */
                           /* writes the state once and applies every gate whose    */
                           /* target lies in the pass's tile qubits. Between passes */
                           /* the qubits are relabelled (the paper's non-sequential */
                           /* storage of the state vector, section Non-Sequential   */
                           /* Storage): a pass writes its tile back with the next   */
                           /* gates' qubits in the low index bits every tile must   */
                           /* hold. The state is in the standard order again when   */
                           /* the call's work completes                             */
#define SV_FUSE_DENSE  2u  /* group gates into dense 2^k x 2^k blocks on k <= 5      */
                           /* qubits, multiplied on the matrix cores (MFMA)          */
#define SV_GRAPH       4u  /* capture the call's launches in a HIP graph once and   */
                           /* replay it when the same gate list (and flags) comes   */
                           /* back (sv_run_circuit), or the same batch request      */
                           /* (sv_batch_run, see there)                              */
#define SV_NO_RELABEL  8u  /* with SV_FUSE: keep the standard storage order between */
                           /* passes (qubits 0..2, or 0..3 for complex64, in every  */
                           /* tile)                                                  */
#define SV_JIT        16u  /* with SV_FUSE: run each pass with a kernel compiled at */
                           /* run time (hipRTC) for that pass's program: its ops'   */
                           /* kinds and register positions fixed in the code, the   */
                           /* numbers still read from the plan. The first call of a */
                           /* program shape compiles it (about a second; passes in  */
                           /* parallel); kernels are kept for the process. Same     */
                           /* arithmetic as the generic pass kernel                  */

/* ABI version; bumped when a signature or struct changes. */
int sv_version(void);

/* Thread-local message of the last failed call ("" when none). The pointer is
 * valid until the next call on the same thread. */
const char *sv_last_error(void);

/* Allocates a 2^n_qubits state in device memory on the current HIP device,
 * owned by the handle, and sets it to |0...0> (the register's starting state).
 * hip_stream: a hipStream_t, or NULL for the null stream. The handle owns the
 * memory until sv_destroy. SV_ENOMEM if hipMalloc fails. */
sv_status sv_create(int n_qubits, sv_dtype dtype, void *hip_stream, sv_state *out);

/* Wraps caller-owned device memory of 2^n_qubits amplitudes (e.g. a torch
 * tensor's data_ptr()). The contents are left as they are. The caller keeps
 * the memory alive until sv_destroy, which does not free it. dev_ptr must be
 * 16-byte aligned. */
sv_status sv_wrap(void *dev_ptr, int n_qubits, sv_dtype dtype, void *hip_stream,
                  sv_state *out);

/* Releases the handle, its scratch buffers and (for sv_create) its state.
 * Waits for the handle's stream first. NULL is accepted. */
sv_status sv_destroy(sv_state s);

/* Changes the stream later calls enqueue on. The caller orders any work
 * already queued on the old stream. */
sv_status sv_set_stream(sv_state s, void *hip_stream);

/* Tile geometry of this handle's SV_FUSE runs and of its plans (the tile pass
 * that applies many gates per sweep of the state; the paper's per-gate sweep,
 * section State Vector Partitioning, is the special case of one gate per
 * sweep). tile_qubits: qubits a pass holds, 4..12 (0: the default, 12);
 * register_qubits: qubits a thread holds in registers per group, 3 or 4 (0:
 * the default, 4; plans always use 4); low_qubits: index bits every tile
 * holds, 0..11 (-1: the default, 3 for complex128 and 4 for complex64; for a
 * state larger than the 256 MiB last-level cache the planner also plans with 6
 * and keeps that plan when it needs no more passes, for longer contiguous
 * runs). All are clamped to the state's qubit count (low_qubits to the tile
 * width minus one). A tuning setting: results depend on
 * it only through the order of rounding (the grouping of gates changes).
 * Drops the handle's captured SV_GRAPH circuit. SV_EINVAL outside the ranges;
 * the setting is then unchanged. */
sv_status sv_set_tile_geometry(sv_state s, int32_t tile_qubits, int32_t register_qubits,
                               int32_t low_qubits);

/* Device pointer, qubit count and dtype of a handle (any out may be NULL). */
sv_status sv_info(sv_state s, void **dev_ptr, int *n_qubits, sv_dtype *dtype);

/* Sets the state to the basis state |basis_index> (basis_index < 2^n). */
sv_status sv_reset(sv_state s, uint64_t basis_index);

/* Sets the state to the uniform superposition 2^{-n/2} sum_x |x>: H on every
 * qubit of |0...0> (section Quantum Information Processing), written in one
 * pass instead of n gate passes. */
sv_status sv_reset_uniform(sv_state s);

/* Applies the 2x2 matrix m to qubit `target`: the stride update of section
 * State Vector Partitioning, one pass over the state. */
sv_status sv_apply_1q(sv_state s, int target, const double m[8]);

/* Applies m to `target` on the amplitudes whose index has bit `control` set
 * (caption of Algorithm 1). control != target. CNOT is m = X; a controlled
 * phase is m = diag(1, e^{i theta}). */
sv_status sv_apply_ctrl(sv_state s, int control, int target, const double m[8]);

/* Applies m to `target` on the amplitudes whose index has every bit of
 * control_mask set: the controlled update with several controls (the Toffoli,
 * or controlled-controlled-NOT, gate of section Quantum Circuits is m = X with
 * two). control_mask must be non-zero, below 2^n and must not hold `target`.
 * One pass over the amplitudes whose control bits are all set. */
sv_status sv_apply_mcu(sv_state s, uint64_t control_mask, int target, const double m[8]);

/* Applies a general gate on k qubits, 1 <= k <= 5: the 2^k x 2^k complex
 * matrix u (row major, (re, im) interleaved FP64, 2 * 4^k doubles, read during
 * the call) acting on the factor of qubits[0..k-1] in the tensor product of
 * section Quantum Information Processing. For every setting of the other index
 * bits, the amplitudes a_c, c = sum_m b_{qubits[m]} 2^m, become
 * sum_c u[r][c] a_c, so qubits[0] is the least significant bit of the local
 * index (u = B (x) A applies A to qubits[0] and B to qubits[1]). The qubits
 * must be distinct and in [0, n); u is not checked for unitarity. k = 1 is
 * sv_apply_1q. For k >= 2 and n >= 9 the gate is one dense 5-qubit block on
 * the matrix cores (u padded with the identity on unused high qubits; one pass
 * over the state); below 9 qubits a small-register kernel applies it. Errors:
 * SV_EINVAL for a null pointer, k out of range, a repeated or out-of-range
 * qubit. */
sv_status sv_apply_unitary(sv_state s, const int32_t *qubits, int32_t k, const double *u);

/* Controlled phase diag(1, e^{i theta}) on (control, target); symmetric in the
 * two qubits. The phase e^{i theta} is formed in FP64 for both dtypes. */
sv_status sv_apply_cphase(sv_state s, int control, int target, double theta);

/* Applies n_gates gates in order (the circuit of section Quantum Circuits).
 * The gate array is read during the call only. flags: 0, SV_FUSE (optionally
 * | SV_NO_RELABEL) or SV_FUSE_DENSE, each optionally | SV_GRAPH. Fusion
 * reorders only gates that act on disjoint qubits, so the result equals the
 * in-order product up to rounding. All gates are validated before any work is
 * queued. Gates with several controls (SV_G_MCU) join tile passes like any
 * other 2x2 (controls in the tile are tested per amplitude, controls outside
 * it per tile); with SV_FUSE_DENSE, one of at most five qubits joins a dense
 * block and a wider one runs as its own launch.
 * SV_GRAPH: the first call plans the list, uploads what its kernels read into
 * buffers of its own and captures the launches (no copies, no memsets) in a
 * HIP graph held by the handle; a later call with the same gate list (compared
 * byte for byte) and the same other flags replays that graph on the handle's
 * stream, with no planning and one host launch. The results are bit for bit
 * those of the same flags without SV_GRAPH. One graph is kept per handle: a
 * different list or flags wait for the handle's earlier replays, free the old
 * graph and capture anew. sv_destroy frees it. */
sv_status sv_run_circuit(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags);

/* sv_run_circuit for gate lists that also hold general k-qubit gates
 * (SV_G_UNITARY records): mats is a table of n_mats matrices, entry j at
 * mats + 2048 j (2 * 32 * 32 doubles; a k-qubit gate uses the first 2 * 4^k,
 * its 2^k x 2^k complex matrix row major, (re, im) interleaved), read during
 * the call only. Each such gate runs as sv_apply_unitary would, between the
 * planned segments of the other gates (list order is kept). SV_GRAPH does not
 * take such records (SV_EUNSUPPORTED). With mats = NULL and n_mats = 0 this is
 * sv_run_circuit. SV_EINVAL for a record with a bad qubit list or a matrix
 * index at or above n_mats. */
sv_status sv_run_circuit_ex(sv_state s, const sv_gate *gates, size_t n_gates, const double *mats,
                            size_t n_mats, uint32_t flags);

/* Runs count independent circuits, circuits[c] (lens[c] gates) on states[c],
 * with their work overlapping on the device: the circuit of section Quantum
 * Circuits applied to many registers at once. Each result equals
 * sv_run_circuit(states[c], circuits[c], lens[c], SV_FUSE) bit for bit.
 * States must be distinct and may mix dtypes, sizes and streams. Circuits on
 * n >= 4 qubits go into one batch per dtype
 * (see sv_batch_run: default launch configuration, circuits of 4096 tiles per
 * pass and more, n >= 24, pass by pass as sv_batch_solo), queued on the stream of
 * that dtype's first such state after the earlier work of every member's
 * stream; the others run alone with SV_FUSE. flags: 0, SV_FUSE (the same) and
 * optionally SV_GRAPH (each batch captured and replayed). Synchronous: returns
 * once every circuit has run. Every state, gate array and gate is validated
 * before any work is queued, so SV_EINVAL leaves all states untouched. For
 * repeated batches, plan once with sv_plan_create and run sv_batch_run. */
sv_status sv_run_batch(sv_state *states, const sv_gate *const *circuits, const size_t *lens,
                       size_t count, uint32_t flags);

/* p_i = |alpha_i|^2 for i in [first, first + count), written to host memory
 * out_host (count doubles). Synchronous: waits for the stream. The squares are
 * formed in FP64 for both dtypes. */
sv_status sv_probs(sv_state s, uint64_t first, uint64_t count, double *out_host);

/* As sv_probs, but writes to device memory out_dev (count doubles, 8-byte
 * aligned) and returns without waiting. */
sv_status sv_probs_device(sv_state s, uint64_t first, uint64_t count, double *out_dev);

/* sum_i |alpha_i|^2 accumulated in FP64 by a fixed two-level tree (the same
 * result bit for bit on every call for the same state). Synchronous. */
sv_status sv_norm(sv_state s, double *out);

/* As sv_norm, but writes the double to device memory and returns without
 * waiting. */
sv_status sv_norm_device(sv_state s, double *out_dev);

/* The error of state a against state b on the GPU, in FP64 (the error
 * statement of a complex64 result against complex128: its largest amplitude
 * error and its norm, the normalisation of section Quantum Information
 * Processing): out[0] = max_i |a_i - b_i| (complex modulus), out[1] =
 * sum_i |a_i - b_i|^2, out[2] = sum_i |a_i|^2, out[3] = sum_i |b_i|^2.
 * Either state may be complex64 or complex128: amplitudes are widened to FP64
 * before they are subtracted. The relative 2-norm error is
 * sqrt(out[1] / out[3]) and a's norm drift |out[2] - 1|. Both states must
 * have the same qubit count and device (SV_EINVAL otherwise). The comparison
 * is queued on a's stream after the work queued so far on b's stream; the call
 * waits for it (synchronous) and allocates 4100 doubles of device scratch for
 * its duration. Both states are read once; the sums use a fixed reduction
 * tree (the same bits on every call). */
sv_status sv_compare(sv_state a, sv_state b, double out[4]);

/* Copies the whole state (2^n amplitudes in the layout above) to / from host
 * memory. Synchronous. */
sv_status sv_copy_out(sv_state s, void *host_dst);
sv_status sv_copy_in(sv_state s, const void *host_src);

/* Waits for the handle's stream; SV_EDEVICE if queued work failed. */
sv_status sv_synchronize(sv_state s);

/* Measurement sampling: draws basis indices with probability |alpha_j|^2 /
 * norm (the measurement of section Quantum Circuits) by inverting the CDF,
 * CDF(j) = sum_{k <= j} |alpha_k|^2 in FP64 (summed in blocks of 4096
 * amplitudes): out_dev[i] = the j with CDF(j - 1) <= u_dev[i] * norm <
 * CDF(j). u_dev: `count` doubles in device memory, in [0, 1) and ascending
 * (the caller's uniform draws, sorted); other input leaves out_dev
 * unspecified. A u whose product with the norm rounds to the norm or above
 * gets the last index of non-zero probability; a state of norm 0 gives 0.
 * out_dev: `count` uint64 in device memory. Queued on the handle's stream;
 * the first call allocates scratch of about 2^(n-11) doubles (SV_ENOMEM if
 * that fails). Reads the state once, plus once more for the blocks of 4096
 * amplitudes that receive samples. */
sv_status sv_sample_device(sv_state s, const double *u_dev, uint64_t count, uint64_t *out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * draws as sv_sample_device, bit for bit, with no allocation of any kind. Its
 * scratch (block sums and their prefix) is a static device array of
 * 2^19 + 2 doubles (4 MiB) that each GPU the library runs on holds until the
 * process ends; so n must be at most 30 (SV_EINVAL above, with nothing
 * queued). Every call on one GPU shares that array: calls queued on one
 * stream are ordered, but calls that overlap on one GPU (other streams or
 * threads) race and give unspecified draws. Nothing in the array needs to be
 * cleared between calls (each call writes every entry it reads). Arguments,
 * errors and the queueing on the handle's stream are as in sv_sample_device. */
sv_status sv_sample_device_noalloc(sv_state s, const double *u_dev, uint64_t count,
                                   uint64_t *out_dev);

/* ---- planned circuits and batched launches --------------------------------
 * A plan is a circuit fused into tile passes (as SV_FUSE does) and uploaded to
 * the device once; it stays bound to the state it was made for. A batch runs
 * pass ranges of many plans, on distinct states of one dtype, level by level:
 * a level launch applies the next pass of several circuits, all their tiles at
 * once, so independent circuits overlap on the device, and the launch boundary
 * orders a circuit's passes (at most one pass of a circuit per level). Levels
 * take circuits in order of least remaining work (passes left times
 * amplitudes) up to about two rounds of tasks per resident work-group, so
 * small circuits finish early and every launch still fills the device. */
typedef struct sv_plan_s *sv_plan;
typedef struct sv_batch_s *sv_batch;

/* Plans gates for state s (n >= 4) and uploads the plan (synchronous). The
 * gate array is read during the call only. The plan is the one SV_FUSE makes
 * (same passes, same results bit for bit), relabelling included: between two
 * of its passes the state may be stored in another qubit order, and it is in
 * the standard order again after the plan's last pass. Read or change the
 * state only before the first or after the last pass has run. */
sv_status sv_plan_create(sv_state s, const sv_gate *gates, size_t n_gates, sv_plan *out);
/* Frees the plan's device memory (waits for work that may use it). */
sv_status sv_plan_destroy(sv_plan p);
/* Number of passes (sweeps over the state) of the plan. */
sv_status sv_plan_passes(sv_plan p, int32_t *n_passes);
/* Queues passes [first_pass, first_pass + count) of the plan on its state's
 * stream, one kernel launch per pass. */
sv_status sv_run_plan(sv_plan p, int32_t first_pass, int32_t count);

/* A batch workspace for dtype on hip_stream (NULL: null stream). A batch must
 * not run twice at the same time; distinct batches may. */
sv_status sv_batch_create(sv_dtype dtype, void *hip_stream, sv_batch *out);
sv_status sv_batch_destroy(sv_batch b);
/* Tuning: work-groups per CU of each level launch (1..8) and tiles per task
 * (1..4096); defaults 3 and 4 for complex64, 2 and 8 for complex128. */
sv_status sv_batch_config(sv_batch b, int32_t blocks_per_cu, int32_t tiles_per_task);
/* Persistent launch for small circuits: a circuit whose passes have at most
 * max_tiles tiles (2^(n-12) for n > 12, one below) runs whole, every pass in
 * order, on one work-group (work-group w takes circuits w, w + G, ..., least
 * work first); one launch covers all of them and runs on a second stream of
 * the batch, beside the levels of the larger circuits (forked from and joined
 * back into the batch stream; captured with them under SV_GRAPH). No
 * work-group ever waits for another (between passes a work-group only fences
 * its own stores and meets its own waves). Results are bit for bit those of the
 * level launches. max_tiles = 0 (the default) turns it off; at most 2^20. */
sv_status sv_batch_persist(sv_batch b, int32_t max_tiles);
/* Large circuits: a circuit whose passes have at least min_tiles tiles (and
 * that the persistent launch does not take) runs pass by pass, one
 * single-state launch per pass as sv_run_plan queues it (each such pass fills
 * the device on its own), on a third stream of the batch, beside the levels
 * and the persistent launch; these circuits run one after another, least work
 * first, and their clocks for sv_batch_times are stamped before the first and
 * after the last pass. Results are bit for bit those of the level launches.
 * min_tiles = 0 (the default) turns it off. */
sv_status sv_batch_solo(sv_batch b, int32_t min_tiles);
/* Queues passes [first_pass[i], first_pass[i] + pass_count[i]) of plans[i],
 * i < count, on the batch's stream (first_pass NULL: from 0; pass_count NULL:
 * to the end). The plans' states must be distinct and of the batch's dtype;
 * their own streams are not used, so the caller orders the batch stream after
 * earlier work on those states. flags: 0 or SV_GRAPH (the level launches are
 * captured in a HIP graph once per identical request and replayed). */
sv_status sv_batch_run(sv_batch b, const sv_plan *plans, const int32_t *first_pass,
                       const int32_t *pass_count, size_t count, uint32_t flags);
/* Waits for the batch stream and writes, for each circuit of the last run,
 * the device-clock times (ms) at which its first tile task started and its
 * last one ended, relative to the earliest start (0 for a circuit with no
 * passes in the run). count must equal that run's. */
sv_status sv_batch_times(sv_batch b, double *start_ms, double *end_ms, size_t count);

/* Plans a gate list for SV_FUSE on the host only (no device is touched) and
 * reports its shape: *n_passes sweeps over the state, *n_groups register
 * groups, *n_ops ops in execution order; gate_op[i] (n_gates entries, or
 * NULL) receives the index of the last op that applies gate i. Gates are
 * validated as in sv_run_circuit for an n_qubits register. flags must be
 * SV_FUSE, optionally | SV_NO_RELABEL (passes that restore the standard
 * order count as passes). Any out pointer may be NULL. */
sv_status sv_plan_inspect(int n_qubits, sv_dtype dtype, const sv_gate *gates, size_t n_gates,
                          uint32_t flags, int32_t *gate_op, int32_t *n_passes, int32_t *n_groups,
                          int32_t *n_ops);

/* Plans a gate list for SV_FUSE | SV_JIT on the host only and compiles the
 * kernels of its distinct pass programs with hipRTC, without touching a device
 * and without keeping them: *n_programs (may be NULL) receives how many there
 * are. flags: SV_FUSE | SV_JIT, optionally | SV_NO_RELABEL. SV_EDEVICE with the
 * compiler's log if a program does not compile. */
sv_status sv_plan_jit_check(int n_qubits, sv_dtype dtype, const sv_gate *gates, size_t n_gates,
                            uint32_t flags, int32_t *n_programs);

/* Plans a gate list for SV_FUSE_DENSE on the host only: *n_blocks blocks of
 * five qubits each. For the first `cap` blocks, block_masks[b] (may be NULL)
 * receives the block's five index bits and block_mats (may be NULL; cap*2048
 * doubles) its 32x32 complex matrix, row major, interleaved (re, im); local
 * index bit k of the matrix is the k-th lowest bit of the mask. The gates of
 * the list, applied in order, equal the blocks' matrices applied in order. */
sv_status sv_plan_dense_inspect(int n_qubits, const sv_gate *gates, size_t n_gates,
                                uint64_t *block_masks, double *block_mats, int32_t cap,
                                int32_t *n_blocks);

/* Per-kernel-class timing of the launches this handle queues, measured with
 * HIP events recorded on the handle's stream around each launch. */
typedef struct {
    char name[16];       /* kernel class: "pair", "pair_ctrl", "swap", "diag", ... */
    uint64_t launches;   /* launches timed */
    double total_ms;     /* summed event-to-event time of those launches */
    double bytes;        /* algorithmic bytes they had to read and write */
    double flops;        /* algorithmic floating-point operations */
} sv_prof_entry;

/* enable != 0: waits for the stream, clears earlier records and starts timing
 * every later launch of this handle; enable == 0 stops timing (records are
 * kept for sv_profile_read). */
sv_status sv_profile(sv_state s, int enable);

/* Waits for the stream and writes up to max_entries classes that have at
 * least one timed launch to out; *n_entries receives the number of such
 * classes (which may exceed max_entries). */
sv_status sv_profile_read(sv_state s, sv_prof_entry *out, int max_entries, int *n_entries);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
