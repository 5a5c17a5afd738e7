// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace svk {

// Amplitudes per 16-byte access: one double2 (c128) or two float2 (c64).
constexpr int kChunkBytes = 16;

inline int elem_bytes(sv_dtype dt) { return dt == SV_C64 ? 8 : 16; }
inline int chunk_log2(sv_dtype dt) { return dt == SV_C64 ? 1 : 0; }

// A 2x2 complex matrix in FP64, row major (q11, q12, q21, q22) as (re, im).
struct Mat2 {
    double q[8];
};

// One term of a diagonal run: amplitudes whose index i has (i & mask) == val
// are multiplied by e^{2 pi i turn / 2^64}. Turns add exactly in uint64 and
// wrap modulo one full turn.
struct DiagTerm {
    uint64_t mask;
    uint64_t val;
    uint64_t turn;
};
constexpr int kMaxDiagTerms = 64;

// ---- streaming 16-byte access -----------------------------------------------
// A load or store of one 16-byte chunk, with the nontemporal hint when NT: for
// state passes that touch every line once and are far larger than the caches,
// so the lines stream through instead of displacing others. A launch whose
// lanes read only part of a 128-byte line per access leaves the rest of the
// line to a later access, which the hint would send back to HBM; such
// launches take NT = false.
// States larger than the last-level cache (256 MiB) take the hint: a pass over
// them touches every line once, and the next pass cannot find them in cache.
constexpr uint64_t kStreamBytes = uint64_t(256) << 20;

template <typename V> struct Native16;
template <> struct Native16<float4> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct Native16<double2> { typedef double T __attribute__((ext_vector_type(2))); };

template <bool NT, typename V>
__device__ __forceinline__ V ld16(const V *p)
{
    if constexpr (NT) {
        using N = typename Native16<V>::T;
        const N n = __builtin_nontemporal_load(reinterpret_cast<const N *>(p));
        V v;
        *reinterpret_cast<N *>(&v) = n;
        return v;
    } else {
        return *p;
    }
}

template <bool NT, typename V>
__device__ __forceinline__ void st16(V *p, const V &v)
{
    if constexpr (NT) {
        using N = typename Native16<V>::T;
        __builtin_nontemporal_store(*reinterpret_cast<const N *>(&v), reinterpret_cast<N *>(p));
    } else {
        *p = v;
    }
}

// Work-groups are dealt to the 8 XCDs in turn (work-group b to XCD b mod 8).
// With span = grid / 8, work-group b takes block (b mod 8) span + b / 8, so
// each XCD walks one contiguous eighth of a launch's range (span 0: block b).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t span)
{
    return span ? (b & 7u) * span + (b >> 3) : b;
}

// ---- launchers (kernels_gate.hip) ----------------------------------------
// All take the state pointer, qubit count and stream; they validate nothing.
hipError_t launch_init(void *psi, int n, sv_dtype dt, uint64_t basis, hipStream_t st);
// 2x2 on target t, optionally controlled by c (c < 0: none). swap_only: the
// matrix is X (a pure exchange of the two amplitudes).
hipError_t launch_pair(void *psi, int n, sv_dtype dt, int t, uint64_t cmask, const Mat2 &m,
                       bool swap_only, hipStream_t st);
// Product of the diagonal terms (at most kMaxDiagTerms).
hipError_t launch_diag(void *psi, int n, sv_dtype dt, const DiagTerm *terms, int count,
                       hipStream_t st);

// ---- launchers (kernels_reduce.hip) --------------------------------------
constexpr int kNormBlocks = 1024;
// partials: kNormBlocks doubles of device scratch; out_dev: one double.
hipError_t launch_norm(const void *psi, int n, sv_dtype dt, double *partials,
                       double *out_dev, hipStream_t st);
hipError_t launch_probs(const void *psi, sv_dtype dt, uint64_t first, uint64_t count,
                        double *out_dev, hipStream_t st);
// States a and b of n qubits (n >= 1), each of either dtype, compared in FP64.
// scratch: 4 * kNormBlocks + 4 doubles; the last four receive max |a_i - b_i|,
// sum |a_i - b_i|^2, sum |a_i|^2 and sum |b_i|^2.
constexpr int kCompareScratch = 4 * kNormBlocks + 4;
hipError_t launch_compare(const void *a, sv_dtype da, const void *b, sv_dtype db, int n,
                          double *scratch, hipStream_t st);

// ---- host helpers (sv_api.hip) ---------------------------------------------
// Records `msg` as the calling thread's last error and returns `st`.
sv_status set_error(sv_status st, const std::string &msg);
uint64_t angle_to_turn(double theta);     // theta radians -> turns * 2^64 (mod 2^64)
bool is_pauli_x(const double m[8]);
bool is_phase_diag(const double m[8]);    // diag(1, e^{i phi}) with |e^{i phi}| == 1

// ---- per-launch timing (profile.hip) ---------------------------------------
// Kernel classes reported by sv_profile_read, in this order.
enum KernelClass {
    KC_INIT = 0, KC_PAIR, KC_PAIR_CTRL, KC_SWAP, KC_DIAG, KC_TILE, KC_DENSE, KC_NORM,
    KC_PROBS, KC_BATCH, KC_SAMPLE, KC_GRAPH, KC_COUNT
};
const char *class_name(int cls);

struct ProfRec {
    int cls;
    double bytes;            // algorithmic bytes moved by the launch
    double flops;            // algorithmic floating-point operations
    hipEvent_t start, stop;
};

struct Profiler {
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
};

}  // namespace svk

namespace svk {
// ---- measurement sampling and the uniform state (kernels_sample.hip) ------
constexpr int kSampleBlockLog = 12;                 // amplitudes per block: 4096
constexpr int kSampleBlock = 1 << kSampleBlockLog;
// Doubles of scratch sampling needs: the block sums, their exclusive prefix
// with the norm at its end, and the index of the last non-zero block.
constexpr uint64_t sample_scratch_doubles(int n)
{
    return 2 * (n < kSampleBlockLog ? uint64_t(1) : (uint64_t(1) << (n - kSampleBlockLog))) + 2;
}
// Largest state the static sampling scratch serves (sv_sample_device_noalloc).
constexpr int kStaticSampleMaxQubits = 30;
// The static sampling scratch of the current device: sample_scratch_doubles(
// kStaticSampleMaxQubits) doubles, held until the process ends. Its device
// address is looked up once per device (the device must be current).
hipError_t static_sample_scratch(int device, double **out);
// S: sample_scratch_doubles(n) doubles of device scratch.
hipError_t launch_block_sums(const void *psi, int n, sv_dtype dt, double *S, hipStream_t st);
// u: m ascending doubles in [0, 1) (device); out: m indices (device).
hipError_t launch_sample(const void *psi, int n, sv_dtype dt, const double *S, const double *u,
                         uint64_t m, uint64_t *out, hipStream_t st);
// Every amplitude set to (value, 0).
hipError_t launch_fill(void *psi, int n, sv_dtype dt, double value, hipStream_t st);
}  // namespace svk

struct sv_state_s {
    void *psi = nullptr;
    int n = 0;
    sv_dtype dt = SV_C128;
    hipStream_t stream = nullptr;
    bool owned = false;
    int device = 0;
    double *scratch = nullptr;        // kNormBlocks + 1 doubles (norm partials + result)
    double *sample_scratch = nullptr; // sampling scratch, allocated on first use
    uint64_t sample_cap = 0;          // its size in doubles
    svk::Profiler prof;
    void *plan = nullptr;             // planner buffers (plan.hip)
    void *graph = nullptr;            // captured circuit graph (graph.hip)
    // Tile geometry of SV_FUSE runs and plans (sv_set_tile_geometry): tile
    // qubits, register qubits, fixed low index bits; 0 / 0 / -1: defaults.
    int tile_L = 0, tile_K = 0, tile_nlow = -1;
};

namespace svk {
// Records a start event when profiling is on; returns a token for prof_end.
int prof_begin(sv_state s);
// Records the stop event of `token` (no-op for -1) with the launch's class,
// algorithmic bytes and flops.
void prof_end(sv_state s, int token, int cls, double bytes, double flops);
void prof_release(sv_state s);
}  // namespace svk
