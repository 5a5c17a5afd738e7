// Device-visible description of a fused tile pass (built by the planner,
// executed by k_tile).
//
// A pass fixes a set T of L "tile" qubits. Work-group g owns the 2^L
// amplitudes whose index bits outside T equal the bits of g; it loads them
// into LDS, applies a program of ops, and writes them back, so the pass costs
// one read and one write of the state however many gates it holds. The
// program is a list of groups; in a group each thread holds 2^K amplitudes
// in registers (the K tile bits S of the group enumerated, the other L-K tile
// bits fixed by the thread id), so every op whose target is in S is applied
// in registers, with one LDS exchange per group.
#pragma once

#ifdef __HIPCC_RTC__
// Compiled at run time (jit.hip): the fixed-width integer types live in the
// run-time compiler's own namespace.
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint8_t uint8_t;
#else
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#endif

namespace svk {

constexpr int kTileMaxL = 13;     // tile bits (c128 and c64: 12)
constexpr int kTileMaxK = 4;      // register bits per group
constexpr int kTileL128 = 12, kTileK128 = 4;   // 64 KiB of complex128 per tile, 256 threads
constexpr int kTileL64 = 12, kTileK64 = 4;     // 32 KiB of complex64 per tile, 256 threads
constexpr int kTileThreads = 512;              // upper bound of 2^(L-K)

enum TileOpKind : int32_t { TOP_U = 0, TOP_SWAP = 1, TOP_DIAG = 2, TOP_U4 = 3 };

// LDS slots that hold a tile of `size` amplitudes: local index l sits in slot
// l + l/32 (complex64) or l + l/16 + l/256 (complex128); the padding keeps
// the accesses of a register group free of bank conflicts.
constexpr uint32_t tile_slots(bool c64, uint32_t size)
{
    return c64 ? size + (size >> 5) : size + (size >> 4) + (size >> 8);
}
constexpr uint32_t kDiagBase = 1u << 31;   // TileOp.dlin: base can be non-zero

// A diagonal op multiplies each amplitude by e^{2 pi i T / 2^64}, where T is
// an exact uint64 sum (mod one full turn): a quadratic form in the index bits,
//     T(i) = sum_q a_q x_q + sum_{q<q'} Q_qq' x_q x_q'      (x_q = bit q of i).
// Controlled-phase gates give the Q terms and one-qubit phases
// diag(1, e^{i phi}) the a terms. The planner never puts a pair term on two
// qubits outside the tile into a pass. In a group, the tile bits are either
// register bits S (k < K) or thread bits (the other L-K, fixed by the thread
// id), and bits outside the tile are fixed by the tile index g, so
//     T = base(tid, g) + sum_{k in r} coef_k(tid, g) + PR(r)
// for the register combination r, with
//     base   = thr[tid][0] + C(g) + sum_{thread bits t set in tid} OW_t(g)
//     coef_k = thr[tid][1 + k] + OW_{s_k}(g)
// where thr holds the tile-independent part of each thread, OW_l(g) the
// weights between tile bit l and the set bits of g, and C(g) the one-qubit
// phases on bits outside the tile. OW and C are sums of byte-table entries,
// one per byte of g: tab[(b * (L + 1) + l) * 256 + byte_b(g)] (l = L is C).
// PR(r), the terms on register bits only, is a constant per op.
struct TileOp {
    int32_t kind;
    int32_t pj;        // TOP_U / TOP_SWAP: target as a position in the group's S;
                       // TOP_U4: the lower of its two positions;
                       // TOP_DIAG: 1 if PR is not zero for every r
    int32_t lctrl;     // control as a local tile bit, or -1
    int32_t octrl;     // control as a global index bit outside the tile, or -1
    int32_t pk;        // TOP_U4: the higher of its two positions;
                       // TOP_U / TOP_SWAP: the control's position in the
                       // group's S when it is a register bit, else -1
    int32_t dthr;      // TOP_DIAG: offset (uint64 units) in the plan's table
                       // area of thr, 2^(L-K) rows of K+1 values
    int32_t dout;      // TOP_DIAG: offset of the byte tables, or -1 (none)
    int32_t dbytes;    // TOP_DIAG: bytes of g the byte tables cover
    // TOP_U / TOP_SWAP with several controls (a Toffoli gate has two): the op
    // applies where every control is 1. lcm: the controls that are tile bits,
    // as a mask of local tile bits (lctrl's bit included; pk is then -1);
    // ocm: the controls outside the tile, as a mask of global index bits
    // (octrl's bit included). Both 0 for ops with at most one control.
    uint32_t lcm;
    // TOP_DIAG: bit k (k < K) set when coef_k can be non-zero for some thread
    // or tile, kDiagBase when base can; the others are zero for every
    // amplitude (a pass compiled for its program skips their phases).
    uint32_t dlin;
    uint64_t ocm;
    double m[8];       // 2x2 in FP64
    float mf[8];       // the same rounded to FP32 (complex64 states)
    double m4[32];     // TOP_U4: 4x4 in FP64, row major, (re, im); basis index
                       // b0 + 2 b1 with b0 the bit at position pj, b1 at pk.
                       // TOP_DIAG: e^{2 pi i PR(r) / 2^64}, r < 16, (re, im)
    float mf4[32];     // the same rounded to FP32
};

struct TileGroup {
    int32_t s[kTileMaxK];          // local tile bits held in registers, ascending
    int32_t ns[kTileMaxL];         // the other L-K local bits: thread bit k is local bit ns[k]
    int32_t op0, nops;
    // Exchanges (X, CNOT) on register bits that end the group are not ops:
    // the write-back sends register combination r to position
    // x(r) = xb ^ (xor of xs[k] over the set bits k of r), an affine map on
    // the K register positions (has_exit = 0: x(r) = r).
    int32_t has_exit;
    uint32_t xb;
    uint32_t xs[kTileMaxK];
};

struct TileArgs {
    void *psi;
    const TileGroup *groups;
    const TileOp *ops;
    const uint64_t *dtab;          // diagonal-op tables (TileOp.dthr, dout)
    const void *phase_tab;         // e^{2 pi i k/256} then e^{2 pi i k/65536}, k < 256
    uint64_t tmask;                // index bits of the tile (L of them)
    uint64_t omask;                // the other index bits of the register
    uint64_t ntiles;               // 2^nnon
    int32_t L;                     // tile bits
    int32_t nlow;                  // tile bits 0..nlow-1 are index bits 0..nlow-1
    int32_t nnon;                  // index bits outside the tile
    int32_t group0, ngroups;
    int32_t has_diag;              // the pass holds diagonal ops (load phase_tab)
    int32_t permute;               // the tile is written back in another qubit order:
    uint64_t osrc;                 // output local bit j takes input local bit
                                   // (osrc >> 4 j) & 15
};

#ifndef __HIPCC_RTC__
// Dynamic LDS of one work-group: padded tile plus the phase table.
size_t tile_lds_bytes(bool c64, int L, bool diag);
// Launches one pass: 2^(L-K) threads per work-group; each work-group walks
// tiles g = blockIdx.x, blockIdx.x + gridDim.x, ... below 2^nnon.
hipError_t launch_tile(const TileArgs &a, int K, bool c64, hipStream_t st);
#endif

// One task of a batched level launch: tiles [tile0, tile0 + ntiles) of pass
// `pass` (an index into BatchArgs.passes) of circuit `circ`.
struct BatchTask {
    int32_t pass;
    int32_t circ;
    uint32_t tile0;
    uint32_t ntiles;
};

struct BatchArgs {
    const BatchTask *tasks;     // all levels, level by level
    const TileArgs *passes;     // tile geometry K = 4 for every pass
    uint64_t *t_start;          // per task: device clock when it started
    uint64_t *t_end;            // per task: device clock when it ended
    uint32_t task0, task_end;   // the tasks of this launch's level
};

// One level of a batch: 2^(L-4) threads per work-group (the largest tile of
// the dtype), blocks_per_cu work-groups per CU taking tasks round-robin.
#ifndef __HIPCC_RTC__
hipError_t launch_level(const BatchArgs &b, bool c64, int blocks_per_cu, hipStream_t st);
#endif

// One circuit of a persistent launch: passes [pass0, pass0 + npass) of
// PersistArgs.passes, all run in order by the one work-group that takes it.
struct PersistCircuit {
    int32_t pass0, npass;
};

// A persistent launch over small circuits: work-group w runs circuits w,
// w + G, ... (G work-groups), all passes of each, every tile of each pass,
// with a fence and a work-group barrier between passes. No work-group waits
// for another; each leaves after its last circuit.
struct PersistArgs {
    const PersistCircuit *circs;
    const TileArgs *passes;
    uint64_t *t_start;          // per circuit: device clock when its first pass started
    uint64_t *t_end;            // per circuit: when its last pass ended
    uint32_t count;
};
#ifndef __HIPCC_RTC__
hipError_t launch_persist(const PersistArgs &p, bool c64, int blocks_per_cu, hipStream_t st);
#endif

}  // namespace svk
