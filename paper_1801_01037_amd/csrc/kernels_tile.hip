// Fused tile pass: one read and one write of the state for a whole run of
// gates (the single-gate stride update of State Vector Partitioning, applied
// many times while the amplitudes sit in LDS and registers).
//
// Work-group g loads the 2^L amplitudes of its tile (index bits outside the
// tile qubits T fixed to the bits of g) into LDS. For each group of ops, each
// thread pulls the 2^K amplitudes that differ in the group's register bits S
// into registers, applies every op of the group there (pair updates on a
// target in S; controls anywhere; diagonal phases), and puts them back. The
// tile is then written to its original place. LDS slots are padded by one
// element every 256 bytes so that register gathers with large local strides
// spread over the banks.
#include <type_traits>

#include "sv_internal.h"
#include "tile.h"

namespace svk {

size_t tile_lds_bytes(bool c64, int L, bool diag)
{
    const size_t size = size_t(1) << L;
    const size_t slots = c64 ? size + (size >> 5) : size + (size >> 4);
    const size_t eb = c64 ? 8 : 16;
    return (slots + (diag ? 512 : 0)) * eb;
}

namespace {

// Amplitudes as clang vector types: plain SSA values, so arrays of them that
// live across loop iterations stay in registers.
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef double dv2 __attribute__((ext_vector_type(2)));

// Plan data is read through the constant address space: the loads are
// uniform, become scalar (s_load), and never wait on the vector-memory
// counter that tracks the prefetch of the next tile.
#define SV_CONST __attribute__((address_space(4)))
typedef const SV_CONST TileGroup CGroup;
typedef const SV_CONST TileOp COp;
typedef const SV_CONST TilePivot CPivot;

template <bool C64>
using RealT = std::conditional_t<C64, float, double>;
template <bool C64>
using AmpT = std::conditional_t<C64, fv2, dv2>;

template <bool C64>
__device__ __forceinline__ uint32_t lds_slot(uint32_t l)
{
    return C64 ? l + (l >> 5) : l + (l >> 4);
}

// Scatters the low bits of x, in order, onto the set bits of mask (the
// "parallel deposit" of x into mask). mask is uniform over the work-group, so
// the loop control stays scalar.
__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t mask)
{
    uint64_t out = 0;
    while (mask) {
        const uint64_t low = mask & (~mask + 1);
        out |= (x & 1) ? low : 0;
        x >>= 1;
        mask &= mask - 1;
    }
    return out;
}

template <typename A>
__device__ __forceinline__ A cmul(A x, A y)
{
    A r;
    r.x = x.x * y.x - x.y * y.y;
    r.y = x.x * y.y + x.y * y.x;
    return r;
}

// e^{2 pi i T / 2^64}: the top two bytes of T select table entries
// e^{2 pi i k/256} and e^{2 pi i k/65536}; the remaining 48 bits are an angle
// below 2 pi / 2^16, done by its Taylor series (error < 1e-22 in FP64; in FP32
// the first-order terms are already below the rounding unit).
template <bool C64>
__device__ __forceinline__ AmpT<C64> turn_phase(uint64_t T, const AmpT<C64> *tab)
{
    using A = AmpT<C64>;
    const A e1 = tab[T >> 56];
    const A e2 = tab[256 + ((T >> 48) & 255u)];
    A e3;
    if constexpr (C64) {
        const float x = float(uint32_t((T >> 16) & 0xFFFFFFFFu)) *
                        float(6.283185307179586476925286766559 * 0x1p-48);
        e3 = fv2{1.0f, x};
    } else {
        const double x = double(T & 0xFFFFFFFFFFFFull) *
                         (6.283185307179586476925286766559 * 0x1p-64);
        const double x2 = x * x;
        e3 = dv2{1.0 - x2 * (0.5 - x2 * (1.0 / 24.0)), x * (1.0 - x2 * (1.0 / 6.0))};
    }
    return cmul(cmul(e1, e2), e3);
}

template <bool C64, int K, int PJ, bool SWAP, bool CTRL>
__device__ __forceinline__ void pair_pj(AmpT<C64> (&v)[1 << K], const uint32_t (&li)[1 << K],
                                        COp &op)
{
    using R = RealT<C64>;
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    const int lc = op.lctrl;
    R m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0, m6 = 0, m7 = 0;
    if constexpr (!SWAP) {
        if constexpr (C64) {
            m0 = op.mf[0]; m1 = op.mf[1]; m2 = op.mf[2]; m3 = op.mf[3];
            m4 = op.mf[4]; m5 = op.mf[5]; m6 = op.mf[6]; m7 = op.mf[7];
        } else {
            m0 = op.m[0]; m1 = op.m[1]; m2 = op.m[2]; m3 = op.m[3];
            m4 = op.m[4]; m5 = op.m[5]; m6 = op.m[6]; m7 = op.m[7];
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r & (1 << PJ)) continue;
        constexpr int bit = 1 << PJ;
        const int r1 = r | bit;
        const A a = v[r], b = v[r1];
        A na, nb;
        if constexpr (SWAP) {
            na = b;
            nb = a;
        } else {
            na.x = m0 * a.x - m1 * a.y + m2 * b.x - m3 * b.y;
            na.y = m0 * a.y + m1 * a.x + m2 * b.y + m3 * b.x;
            nb.x = m4 * a.x - m5 * a.y + m6 * b.x - m7 * b.y;
            nb.y = m4 * a.y + m5 * a.x + m6 * b.y + m7 * b.x;
        }
        if constexpr (CTRL) {
            const bool on = (li[r] >> lc) & 1u;
            v[r] = on ? na : a;
            v[r1] = on ? nb : b;
        } else {
            v[r] = na;
            v[r1] = nb;
        }
    }
}

template <bool C64, int K, bool SWAP, bool CTRL>
__device__ __forceinline__ void apply_pair(AmpT<C64> (&v)[1 << K], const uint32_t (&li)[1 << K],
                                           COp &op)
{
    switch (op.pj) {
    case 0: pair_pj<C64, K, 0, SWAP, CTRL>(v, li, op); break;
    case 1: if constexpr (K > 1) pair_pj<C64, K, 1, SWAP, CTRL>(v, li, op); break;
    case 2: if constexpr (K > 2) pair_pj<C64, K, 2, SWAP, CTRL>(v, li, op); break;
    case 3: if constexpr (K > 3) pair_pj<C64, K, 3, SWAP, CTRL>(v, li, op); break;
    default: break;
    }
}

template <bool C64, int K>
__device__ __forceinline__ void apply_diag(AmpT<C64> (&v)[1 << K], const uint32_t (&li)[1 << K],
                                           COp &op, CPivot *pivots, int L,
                                           CGroup &G, uint64_t gbase, uint32_t tid,
                                           const AmpT<C64> *tab)
{
    constexpr int NR = 1 << K;
    uint64_t T[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) T[r] = 0;
    for (int p = 0; p < op.npiv; ++p) {
        CPivot &P = pivots[op.piv0 + p];
        if (P.opivot >= 0 && !((gbase >> P.opivot) & 1ull)) continue;
        uint64_t c = P.w0;
        for (int k = 0; k < P.nout; ++k)
            c += ((gbase >> P.obit[k]) & 1ull) ? P.ow[k] : 0ull;
        for (int k = 0; k < L - K; ++k)
            c += ((tid >> k) & 1u) ? P.wl[G.ns[k]] : 0ull;
        uint64_t ws[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ws[k] = P.wl[G.s[k]];
        const int lp = P.lpivot;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            uint64_t t = c;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (r & (1 << k)) t += ws[k];
            const bool on = lp < 0 || ((li[r] >> lp) & 1u);
            T[r] += on ? t : 0ull;
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (T[r] != 0) v[r] = cmul(v[r], turn_phase<C64>(T[r], tab));
}

// One work-group walks tiles blockIdx.x, +gridDim.x, ...; the next tile's
// amplitudes are loaded into registers while the current one is processed.
template <bool C64, int K, bool PREF>
__device__ __forceinline__ void tile_body(const TileArgs a)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    extern __shared__ __align__(16) unsigned char smem[];
    A *lds = reinterpret_cast<A *>(smem);
    const uint32_t size = 1u << a.L;
    const uint32_t slots = C64 ? size + (size >> 5) : size + (size >> 4);
    A *tab = lds + slots;
    const uint32_t W = 1u << (a.L - K);
    const uint32_t tid = threadIdx.x;
    A *psi = static_cast<A *>(a.psi);

    if (a.has_diag) {
        const A *src = static_cast<const A *>(a.phase_tab);
        for (uint32_t i = tid; i < 512; i += W) tab[i] = src[i];
    }
    CGroup *groups = (CGroup *)(a.groups);
    COp *ops = (COp *)(a.ops);
    CPivot *pivots = (CPivot *)(a.pivots);
    const uint64_t dt = deposit(tid, a.tmask);
    uint64_t roff[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) roff[r] = deposit(uint64_t(r) * W, a.tmask);

    uint64_t g = blockIdx.x;
    A pv[NR];
    if (PREF && g < a.ntiles) {
        const uint64_t gb = deposit(g, a.omask) | dt;
#pragma unroll
        for (int r = 0; r < NR; ++r) pv[r] = psi[gb | roff[r]];
    }
    while (g < a.ntiles) {
        const uint64_t gbase = deposit(g, a.omask);
        if (!PREF) {
#pragma unroll
            for (int r = 0; r < NR; ++r) pv[r] = psi[gbase | dt | roff[r]];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(tid + uint32_t(r) * W)] = pv[r];
        __syncthreads();
        const uint64_t gn = g + gridDim.x;
        if (PREF && gn < a.ntiles) {
            const uint64_t gb = deposit(gn, a.omask) | dt;
#pragma unroll
            for (int r = 0; r < NR; ++r) pv[r] = psi[gb | roff[r]];
        }
        for (int gi = 0; gi < a.ngroups; ++gi) {
            CGroup &G = groups[a.group0 + gi];
            uint32_t lbase = 0;
            for (int k = 0; k < a.L - K; ++k) lbase |= ((tid >> k) & 1u) << G.ns[k];
            uint32_t soff[K];
#pragma unroll
            for (int k = 0; k < K; ++k) soff[k] = 1u << G.s[k];
            uint32_t li[NR];
            A v[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                uint32_t l = lbase;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (r & (1 << k)) l |= soff[k];
                li[r] = l;
                v[r] = lds[lds_slot<C64>(l)];
            }
            for (int oi = 0; oi < G.nops; ++oi) {
                COp &op = ops[G.op0 + oi];
                if (op.kind == TOP_DIAG) {
                    apply_diag<C64, K>(v, li, op, pivots, a.L, G, gbase, tid, tab);
                    continue;
                }
                if (op.octrl >= 0 && !((gbase >> op.octrl) & 1ull)) continue;
                const bool ctrl = op.lctrl >= 0;
                if (op.kind == TOP_SWAP) {
                    if (ctrl) apply_pair<C64, K, true, true>(v, li, op);
                    else apply_pair<C64, K, true, false>(v, li, op);
                } else {
                    if (ctrl) apply_pair<C64, K, false, true>(v, li, op);
                    else apply_pair<C64, K, false, false>(v, li, op);
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(li[r])] = v[r];
            __syncthreads();
        }
        // Each thread stores the slots it filled, so the next fill needs no barrier.
        const uint64_t gb = gbase | dt;
#pragma unroll
        for (int r = 0; r < NR; ++r) psi[gb | roff[r]] = lds[lds_slot<C64>(tid + uint32_t(r) * W)];
        g = gn;
    }
}

// One kernel per (dtype, register bits K, prefetch) with at most MAXT threads.
template <bool C64, int K, bool PREF, int MAXT>
__global__ __launch_bounds__(MAXT) void k_tile(TileArgs a)
{
    tile_body<C64, K, PREF>(a);
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
hipError_t launch_k(Kern kern, bool c64, const TileArgs &a, int K, size_t lds, hipStream_t st)
{
    // Allow the largest tile this dtype uses (above the 64 KiB default).
    const int max_lds = int(tile_lds_bytes(c64, c64 ? kTileL64 : kTileL128, true));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e != hipSuccess) return e;
    const uint64_t want = uint64_t(cu_count()) * 2;
    const unsigned grid = unsigned(a.ntiles < want ? a.ntiles : want);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1u << (a.L - K)), lds, st, a);
    return hipGetLastError();
}

template <bool C64, bool PREF>
hipError_t launch_dt(const TileArgs &a, int K, size_t lds, hipStream_t st)
{
    switch (K) {
    case 1: return launch_k(k_tile<C64, 1, PREF, 1024>, C64, a, K, lds, st);
    case 2: return launch_k(k_tile<C64, 2, PREF, 1024>, C64, a, K, lds, st);
    case 3: return launch_k(k_tile<C64, 3, PREF, C64 ? 1024 : 512>, C64, a, K, lds, st);
    case 4: return launch_k(k_tile<C64, 4, PREF, C64 ? 512 : 256>, C64, a, K, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tile(const TileArgs &a, int K, bool c64, bool prefetch, hipStream_t st)
{
    if ((1u << (a.L - K)) > 1024u) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(c64, a.L, a.has_diag != 0);
    if (c64) return prefetch ? launch_dt<true, true>(a, K, lds, st) : launch_dt<true, false>(a, K, lds, st);
    return prefetch ? launch_dt<false, true>(a, K, lds, st) : launch_dt<false, false>(a, K, lds, st);
}

}  // namespace svk
