// Fused tile pass: one read and one write of the state for a whole run of
// gates (the single-gate stride update of State Vector Partitioning, applied
// many times while the amplitudes sit in LDS and registers).
//
// Work-group g loads the 2^L amplitudes of its tile (index bits outside the
// tile qubits T fixed to the bits of g) into LDS. For each group of ops, each
// thread pulls the 2^K amplitudes that differ in the group's register bits S
// into registers, applies every op of the group there (pair updates on a
// target in S; controls anywhere; diagonal phases), and puts them back. The
// tile is then written to its original place, optionally with its qubits in
// another order (the planner's relabelling of storage bits inside the tile,
// which leaves the amplitudes the tile covers unchanged). LDS slots are padded by one
// element every 256 bytes so that register gathers with large local strides
// spread over the banks.
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "sv_internal.h"
#include "tile.h"
#include "tile_dev.h"

namespace svk {

size_t tile_lds_bytes(bool c64, int L, bool diag)
{
    const size_t size = size_t(1) << L;
    const size_t slots = tile_slots(c64, uint32_t(size));
    const size_t eb = c64 ? 8 : 16;
    return (slots + (diag ? 512 : 0)) * eb;
}

namespace {

using namespace dev;

// The generic program of a pass: its groups and ops read from their device
// records and dispatched at run time.
template <bool C64, int K>
struct RecordedGroups {
    const TileArgs &a;
    AmpT<C64> *lds;
    const AmpT<C64> *tab;

    __device__ __forceinline__ void operator()(uint64_t g, uint64_t gbase, const Walk<K> &w,
                                               const Amps<C64, K> &) const
    {
        using A = AmpT<C64>;
        constexpr int NR = 1 << K;
        CGroup *groups = (CGroup *)(a.groups);
        COp *ops = (COp *)(a.ops);
        for (int gi = 0; gi < a.ngroups; ++gi) {
            CGroup &G = groups[a.group0 + gi];
            // Waves applying a group's ops issue ahead of the other work-group's
            // waves that exchange through LDS or move tiles (layered step
            // -1.8 %, QFT -2.5 % for complex128; -1.7 % / -4.4 % complex64).
            __builtin_amdgcn_s_setprio(2);
            if (w.active) {
                uint32_t lbase = 0;
                for (int k = 0; k < a.L - K; ++k) lbase |= ((w.tid >> k) & 1u) << G.ns[k];
                uint32_t soff[K];
#pragma unroll
                for (int k = 0; k < K; ++k) soff[k] = 1u << G.s[k];
                A v[NR], u[NR];
                gather<C64, K>(lds, lbase, soff, v);
                // Ops alternate v -> u and u -> v; the group ends in either.
                // The write-back applies the group's exit exchanges: only this
                // thread's own slots are permuted, so no barrier is needed.
                const int nops = G.nops;
                const bool exit_map = G.has_exit != 0;
                for (int oi = 0;; oi += 2) {
                    if (oi == nops) {
                        scatter<C64, K>(lds, v, lbase, soff, G, exit_map);
                        break;
                    }
                    apply_op<C64, K>(v, u, lbase, soff, ops[G.op0 + oi], a.dtab, a.L, G, g, gbase, w.tid, tab);
                    if (oi + 1 == nops) {
                        scatter<C64, K>(lds, u, lbase, soff, G, exit_map);
                        break;
                    }
                    apply_op<C64, K>(u, v, lbase, soff, ops[G.op0 + oi + 1], a.dtab, a.L, G, g, gbase, w.tid, tab);
                }
            }
            __builtin_amdgcn_s_setprio(0);
            lds_barrier();
        }
    }
};

template <bool C64, int K, bool NT = false>
__device__ __forceinline__ void run_tiles(const TileArgs &a, uint64_t g0, uint64_t gend,
                                          uint64_t gstep, AmpT<C64> *lds, AmpT<C64> *tab)
{
    walk_tiles<C64, K, NT>(a, g0, gend, gstep, lds, tab, RecordedGroups<C64, K>{a, lds, tab},
                           NoFetch{});
}

template <bool C64>
__device__ __forceinline__ AmpT<C64> *lds_base()
{
    extern __shared__ __align__(16) unsigned char smem[];
    return reinterpret_cast<AmpT<C64> *>(smem);
}

// One pass: work-group blockIdx.x walks tiles blockIdx.x, +gridDim.x, ...
template <bool C64, int K, int MAXT, bool NT = false>
__global__ __launch_bounds__(MAXT) void k_tile(TileArgs a)
{
    using A = AmpT<C64>;
    A *lds = lds_base<C64>();
    const uint32_t size = 1u << a.L;
    A *tab = lds + tile_slots(C64, size);
    run_tiles<C64, K, NT>(a, blockIdx.x, a.ntiles, gridDim.x, lds, tab);
}

// One pass level of a batch: every task (a chunk of tiles of one pass of one
// circuit) of the level is independent of the others, so work-groups take
// tasks blockIdx.x, +gridDim.x, ... with no waiting; the launch boundary
// orders consecutive levels of a circuit. Each task stores its start and end
// device clock.
template <bool C64, int MAXT>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(C64 ? 3 : 1)))
void k_level(BatchArgs b)
{
    using A = AmpT<C64>;
    constexpr int K = 4;
    A *lds = lds_base<C64>();
    const BatchTask SV_CONST *tasks = (const BatchTask SV_CONST *)(b.tasks);
    const TileArgs SV_CONST *passes = (const TileArgs SV_CONST *)(b.passes);
    for (uint32_t ti = b.task0 + blockIdx.x; ti < b.task_end; ti += gridDim.x) {
        const BatchTask SV_CONST &t = tasks[ti];
        const uint32_t tile0 = t.tile0, ntiles = t.ntiles;
        const TileArgs SV_CONST &pc = passes[t.pass];
        TileArgs a;
        a.psi = pc.psi; a.groups = pc.groups; a.ops = pc.ops; a.dtab = pc.dtab;
        a.phase_tab = pc.phase_tab; a.tmask = pc.tmask; a.omask = pc.omask; a.ntiles = pc.ntiles;
        a.L = pc.L; a.nlow = pc.nlow; a.nnon = pc.nnon; a.group0 = pc.group0;
        a.ngroups = pc.ngroups; a.has_diag = pc.has_diag; a.permute = pc.permute; a.osrc = pc.osrc;
        if (threadIdx.x == 0) b.t_start[ti] = wall_clock64();
        const uint32_t size = 1u << a.L;
        A *tab = lds + tile_slots(C64, size);
        run_tiles<C64, K>(a, tile0, uint64_t(tile0) + ntiles, 1, lds, tab);
        if (threadIdx.x == 0) b.t_end[ti] = wall_clock64();
        lds_barrier();   // the next task reuses LDS
    }
}

// Persistent launch over whole small circuits (see PersistArgs): work-group
// w runs circuits w, w + G, w + 2G, ... (G work-groups), every pass of each in
// order. The loop index is uniform and its trip count fixed, and no
// work-group waits for another. (Taking circuits from a shared queue counter,
// with one lane doing the atomic add and the index broadcast through LDS,
// made the compiler split this loop around that lane: the other lanes then
// ran the same circuit again without end.)
template <bool C64, int MAXT>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(C64 ? 3 : 1)))
void k_persist(PersistArgs p)
{
    using A = AmpT<C64>;
    constexpr int K = 4;
    A *lds = lds_base<C64>();
    const PersistCircuit SV_CONST *circs = (const PersistCircuit SV_CONST *)(p.circs);
    const TileArgs SV_CONST *passes = (const TileArgs SV_CONST *)(p.passes);
    for (uint32_t c = blockIdx.x; c < p.count; c += gridDim.x) {
        const int32_t pass0 = circs[c].pass0, npass = circs[c].npass;
        if (threadIdx.x == 0) p.t_start[c] = wall_clock64();
        for (int32_t k = 0; k < npass; ++k) {
            const TileArgs SV_CONST &pc = passes[pass0 + k];
            TileArgs a;
            a.psi = pc.psi; a.groups = pc.groups; a.ops = pc.ops; a.dtab = pc.dtab;
            a.phase_tab = pc.phase_tab; a.tmask = pc.tmask; a.omask = pc.omask; a.ntiles = pc.ntiles;
            a.L = pc.L; a.nlow = pc.nlow; a.nnon = pc.nnon; a.group0 = pc.group0;
            a.ngroups = pc.ngroups; a.has_diag = pc.has_diag; a.permute = pc.permute; a.osrc = pc.osrc;
            const uint32_t size = 1u << a.L;
            A *tab = lds + tile_slots(C64, size);
            run_tiles<C64, K>(a, 0, a.ntiles, 1, lds, tab);
            // The next pass loads what this one stored, from other waves of
            // the work-group: release the stores, meet, acquire.
            __threadfence();
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (threadIdx.x == 0) p.t_end[c] = wall_clock64();
    }
}

int cu_count()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

template <typename Kern>
hipError_t set_max_lds(Kern kern, bool c64)
{
    // Allow the largest tile this dtype uses (above the 64 KiB default).
    const int max_lds = int(tile_lds_bytes(c64, c64 ? kTileL64 : kTileL128, true));
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
}

// Work-groups of `kern` that fit on one CU with `threads` threads and `lds`
// bytes of LDS, after raising the kernel's LDS limit. Both are asked of the
// runtime once per (kernel, device, shape) and then kept: a short circuit
// queues many tile launches, and each query costs host time.
template <typename Kern>
hipError_t resident_per_cu(Kern kern, bool c64, int threads, size_t lds, int *per_cu)
{
    using Key = std::tuple<const void *, int, int, size_t>;
    static std::mutex mu;
    static std::map<Key, int> known;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const Key key{reinterpret_cast<const void *>(kern), dev, threads, lds};
    std::lock_guard<std::mutex> lock(mu);
    const auto it = known.find(key);
    if (it != known.end()) {
        *per_cu = it->second;
        return hipSuccess;
    }
    hipError_t e = set_max_lds(kern, c64);
    if (e != hipSuccess) return e;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, lds) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        n = 1;
    }
    known.emplace(key, n);
    *per_cu = n;
    return hipSuccess;
}

template <typename Kern>
hipError_t launch_k(Kern kern, bool c64, const TileArgs &a, int K, size_t lds, hipStream_t st)
{
    // One work-group per resident slot (LDS and registers decide how many
    // fit on a CU); each walks its tiles with a grid stride.
    const int threads = 1 << (a.L - K);
    int per_cu = 1;
    hipError_t e = resident_per_cu(kern, c64, threads, lds, &per_cu);
    if (e != hipSuccess) return e;
    const uint64_t want = uint64_t(cu_count()) * uint64_t(per_cu);
    const unsigned grid = unsigned(a.ntiles < want ? a.ntiles : want);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, a);
    return hipGetLastError();
}

template <bool C64>
hipError_t launch_dt(const TileArgs &a, int K, size_t lds, hipStream_t st)
{
    switch (K) {
    case 1: return launch_k(k_tile<C64, 1, 1024>, C64, a, K, lds, st);
    case 2: return launch_k(k_tile<C64, 2, 1024>, C64, a, K, lds, st);
    case 3: return launch_k(k_tile<C64, 3, C64 ? 1024 : 512>, C64, a, K, lds, st);
    case 4:
        // Only states past the last-level cache stream; they all run K = 4.
        if ((a.ntiles << a.L) * uint64_t(C64 ? 8 : 16) > kStreamBytes)
            return launch_k(k_tile<C64, 4, C64 ? 512 : 256, true>, C64, a, K, lds, st);
        return launch_k(k_tile<C64, 4, C64 ? 512 : 256>, C64, a, K, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_persist(const PersistArgs &p, bool c64, int blocks_per_cu, hipStream_t st)
{
    if (p.count == 0) return hipSuccess;
    const int threads = c64 ? (1 << (kTileL64 - 4)) : (1 << (kTileL128 - 4));
    const size_t lds = tile_lds_bytes(c64, c64 ? kTileL64 : kTileL128, true);
    const uint32_t want = uint32_t(cu_count() * (blocks_per_cu > 0 ? blocks_per_cu : 2));
    const unsigned grid = p.count < want ? p.count : want;
    hipError_t e;
    if (c64) {
        if ((e = set_max_lds(k_persist<true, 256>, true)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_persist<true, 256>), dim3(grid), dim3(threads), lds, st, p);
    } else {
        if ((e = set_max_lds(k_persist<false, 256>, false)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_persist<false, 256>), dim3(grid), dim3(threads), lds, st, p);
    }
    return hipGetLastError();
}

hipError_t launch_tile(const TileArgs &a, int K, bool c64, hipStream_t st)
{
    if ((1u << (a.L - K)) > 1024u) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(c64, a.L, a.has_diag != 0);
    return c64 ? launch_dt<true>(a, K, lds, st) : launch_dt<false>(a, K, lds, st);
}

hipError_t launch_level(const BatchArgs &b, bool c64, int blocks_per_cu, hipStream_t st)
{
    const uint32_t ntasks = b.task_end - b.task0;
    if (ntasks == 0) return hipSuccess;
    const int threads = c64 ? (1 << (kTileL64 - 4)) : (1 << (kTileL128 - 4));
    const size_t lds = tile_lds_bytes(c64, c64 ? kTileL64 : kTileL128, true);
    const uint32_t want = uint32_t(cu_count() * (blocks_per_cu > 0 ? blocks_per_cu : 2));
    const unsigned grid = ntasks < want ? ntasks : want;
    hipError_t e;
    if (c64) {
        if ((e = set_max_lds(k_level<true, 256>, true)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_level<true, 256>), dim3(grid), dim3(threads), lds, st, b);
    } else {
        if ((e = set_max_lds(k_level<false, 256>, false)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_level<false, 256>), dim3(grid), dim3(threads), lds, st, b);
    }
    return hipGetLastError();
}

}  // namespace svk
