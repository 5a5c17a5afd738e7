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
// counter that tracks the tile loads.
#define SV_CONST __attribute__((address_space(4)))
typedef const SV_CONST TileGroup CGroup;
typedef const SV_CONST TileOp COp;
typedef const SV_CONST uint64_t CU64;

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

template <typename R>
__device__ __forceinline__ R fmadd(R a, R b, R c)
{
    if constexpr (std::is_same_v<R, float>) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// Every op reads the amplitudes from `in` and writes all of them to `out`;
// the group loop alternates two arrays, so results never need copying back.
template <bool C64, int K>
using Amps = AmpT<C64>[1 << K];

template <bool C64, int K>
__device__ __forceinline__ void copy_amps(const Amps<C64, K> &in, Amps<C64, K> &out)
{
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) out[r] = in[r];
}

template <bool C64, int K, int PJ, bool SWAP, bool CTRL>
__device__ __forceinline__ void pair_pj(const Amps<C64, K> &in, Amps<C64, K> &out,
                                        const uint32_t (&li)[1 << K], COp &op)
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
        const A a = in[r], b = in[r1];
        A na, nb;
        if constexpr (SWAP) {
            na = b;
            nb = a;
        } else {
            na.x = fmadd(-m3, b.y, fmadd(m2, b.x, fmadd(-m1, a.y, m0 * a.x)));
            na.y = fmadd(m3, b.x, fmadd(m2, b.y, fmadd(m1, a.x, m0 * a.y)));
            nb.x = fmadd(-m7, b.y, fmadd(m6, b.x, fmadd(-m5, a.y, m4 * a.x)));
            nb.y = fmadd(m7, b.x, fmadd(m6, b.y, fmadd(m5, a.x, m4 * a.y)));
        }
        if constexpr (CTRL) {
            const bool on = (li[r] >> lc) & 1u;
            out[r] = on ? na : a;
            out[r1] = on ? nb : b;
        } else {
            out[r] = na;
            out[r1] = nb;
        }
    }
}

template <bool C64, int K, bool SWAP, bool CTRL>
__device__ __forceinline__ void apply_pair(const Amps<C64, K> &in, Amps<C64, K> &out,
                                           const uint32_t (&li)[1 << K], COp &op)
{
    // The planner emits positions below K only; the other arms are unreachable
    // (an arm that wrote nothing, or copied, would keep the other array live or
    // be hoisted in front of every op).
    switch (op.pj) {
    case 0: pair_pj<C64, K, 0, SWAP, CTRL>(in, out, li, op); break;
    case 1:
        if constexpr (K > 1) pair_pj<C64, K, 1, SWAP, CTRL>(in, out, li, op);
        else __builtin_unreachable();
        break;
    case 2:
        if constexpr (K > 2) pair_pj<C64, K, 2, SWAP, CTRL>(in, out, li, op);
        else __builtin_unreachable();
        break;
    case 3:
        if constexpr (K > 3) pair_pj<C64, K, 3, SWAP, CTRL>(in, out, li, op);
        else __builtin_unreachable();
        break;
    default: __builtin_unreachable();
    }
}

// A 2x2 (or an exchange) on register position PJ controlled by register
// position PC: only the pairs whose PC bit is set are updated, the others
// are copied; with both positions fixed at compile time an exchange is a
// plain register permutation.
template <bool C64, int K, int PJ, int PC, bool SWAP>
__device__ __forceinline__ void pair_rc(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op)
{
    using R = RealT<C64>;
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    constexpr int bj = 1 << PJ, bc = 1 << PC;
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
        if (r & bj) continue;
        const int r1 = r | bj;
        if (!(r & bc)) {
            out[r] = in[r];
            out[r1] = in[r1];
            continue;
        }
        const A a = in[r], b = in[r1];
        if constexpr (SWAP) {
            out[r] = b;
            out[r1] = a;
        } else {
            A na, nb;
            na.x = fmadd(-m3, b.y, fmadd(m2, b.x, fmadd(-m1, a.y, m0 * a.x)));
            na.y = fmadd(m3, b.x, fmadd(m2, b.y, fmadd(m1, a.x, m0 * a.y)));
            nb.x = fmadd(-m7, b.y, fmadd(m6, b.x, fmadd(-m5, a.y, m4 * a.x)));
            nb.y = fmadd(m7, b.x, fmadd(m6, b.y, fmadd(m5, a.x, m4 * a.y)));
            out[r] = na;
            out[r1] = nb;
        }
    }
}

template <bool C64, int K, int PJ, bool SWAP>
__device__ __forceinline__ void apply_rc_j(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op)
{
    // The planner sets pk (the control's register position) below K and
    // different from pj; the other arms are unreachable.
    switch (op.pk) {
    case 0:
        if constexpr (PJ != 0) pair_rc<C64, K, PJ, 0, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    case 1:
        if constexpr (K > 1 && PJ != 1) pair_rc<C64, K, PJ, 1, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    case 2:
        if constexpr (K > 2 && PJ != 2) pair_rc<C64, K, PJ, 2, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    case 3:
        if constexpr (K > 3 && PJ != 3) pair_rc<C64, K, PJ, 3, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    default: __builtin_unreachable();
    }
}

template <bool C64, int K, bool SWAP>
__device__ __forceinline__ void apply_rc(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op)
{
    switch (op.pj) {
    case 0: apply_rc_j<C64, K, 0, SWAP>(in, out, op); break;
    case 1:
        if constexpr (K > 1) apply_rc_j<C64, K, 1, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    case 2:
        if constexpr (K > 2) apply_rc_j<C64, K, 2, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    case 3:
        if constexpr (K > 3) apply_rc_j<C64, K, 3, SWAP>(in, out, op);
        else __builtin_unreachable();
        break;
    default: __builtin_unreachable();
    }
}

// A 4x4 unitary on register positions P0 < P1: each quad of amplitudes that
// differ only in those two bits is multiplied by the matrix.
template <bool C64, int K, int P0, int P1>
__device__ __forceinline__ void u4_pp(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op)
{
    using R = RealT<C64>;
    constexpr int NR = 1 << K;
    constexpr int b0 = 1 << P0, b1 = 1 << P1;
    R m[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) m[k] = C64 ? R(op.mf4[k]) : R(op.m4[k]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r & (b0 | b1)) continue;
        const int idx[4] = {r, r | b0, r | b1, r | b0 | b1};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // one FMA chain per real component: re = sum_j Re(m_ij x_j)
            R re = m[8 * i] * in[idx[0]].x;
            R im = m[8 * i] * in[idx[0]].y;
            re = fmadd(-m[8 * i + 1], in[idx[0]].y, re);
            im = fmadd(m[8 * i + 1], in[idx[0]].x, im);
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                const R mr = m[(4 * i + j) * 2], mi = m[(4 * i + j) * 2 + 1];
                re = fmadd(mr, in[idx[j]].x, re);
                re = fmadd(-mi, in[idx[j]].y, re);
                im = fmadd(mr, in[idx[j]].y, im);
                im = fmadd(mi, in[idx[j]].x, im);
            }
            out[idx[i]].x = re;
            out[idx[i]].y = im;
        }
    }
}

template <bool C64, int K>
__device__ __forceinline__ void apply_u4(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op)
{
    const int code = op.pj * 4 + op.pk;
#define SV_U4_CASE(P0, P1)                                                        \
    case P0 * 4 + P1:                                                             \
        if constexpr (K > P1) u4_pp<C64, K, P0, P1>(in, out, op);                 \
        else __builtin_unreachable();                                             \
        break;
    switch (code) {
    SV_U4_CASE(0, 1)
    SV_U4_CASE(0, 2)
    SV_U4_CASE(0, 3)
    SV_U4_CASE(1, 2)
    SV_U4_CASE(1, 3)
    SV_U4_CASE(2, 3)
    default: __builtin_unreachable();   // the planner emits P0 < P1 < K only
    }
#undef SV_U4_CASE
}

// Diagonal op (the quadratic phase form described with TileOp): the turn of
// register combination r is base + sum_{k in r} coef_k + PR(r), so the phase
// of every amplitude is a product of five evaluated phases and a constant.
template <bool C64, int K>
__device__ __forceinline__ void apply_diag(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op,
                                           const uint64_t *dtab, int L, CGroup &G, uint64_t g,
                                           uint32_t tid, const AmpT<C64> *tab)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    const uint64_t *th = dtab + op.dthr + size_t(tid) * (K + 1);
    uint64_t base = th[0];
    uint64_t coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = th[1 + k];
    if (op.dout >= 0) {
        // Weights against the bits of g: uniform byte-table sums (scalar loads).
        CU64 *bt = (CU64 *)(dtab + op.dout);
        auto ow = [&](int l) {
            uint64_t w = 0;
            for (int b = 0; b < op.dbytes; ++b)
                w += bt[(size_t(b) * (L + 1) + l) * 256 + ((g >> (8 * b)) & 255u)];
            return w;
        };
        base += ow(L);
        for (int k = 0; k < L - K; ++k) {
            const uint64_t w = ow(G.ns[k]);
            base += ((tid >> k) & 1u) ? w : 0ull;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) coef[k] += ow(G.s[k]);
    }
    A e[NR];
    A ek[K];
    e[0] = turn_phase<C64>(base, tab);
#pragma unroll
    for (int k = 0; k < K; ++k) ek[k] = turn_phase<C64>(coef[k], tab);
#pragma unroll
    for (int r = 1; r < NR; ++r) {
        const int k = 31 - __builtin_clz(unsigned(r));
        e[r] = cmul(e[r ^ (1 << k)], ek[k]);
    }
    if (op.pj) {   // register-only terms
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            A c;
            if constexpr (C64) { c.x = op.mf4[2 * r]; c.y = op.mf4[2 * r + 1]; }
            else { c.x = op.m4[2 * r]; c.y = op.m4[2 * r + 1]; }
            e[r] = cmul(e[r], c);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r] = cmul(in[r], e[r]);
}

// Applies one op of group G: in -> out.
template <bool C64, int K>
__device__ __forceinline__ void apply_op(const Amps<C64, K> &in, Amps<C64, K> &out,
                                         const uint32_t (&li)[1 << K], COp &op,
                                         const uint64_t *dtab, int L, CGroup &G, uint64_t g,
                                         uint64_t gbase, uint32_t tid, const AmpT<C64> *tab)
{
    if (op.kind == TOP_DIAG) {
        apply_diag<C64, K>(in, out, op, dtab, L, G, g, tid, tab);
    } else if (op.kind == TOP_U4) {
        apply_u4<C64, K>(in, out, op);
    } else if (op.octrl >= 0 && !((gbase >> op.octrl) & 1ull)) {
        copy_amps<C64, K>(in, out);
    } else if (op.kind == TOP_SWAP) {
        if (op.pk >= 0) apply_rc<C64, K, true>(in, out, op);
        else if (op.lctrl >= 0) apply_pair<C64, K, true, true>(in, out, li, op);
        else apply_pair<C64, K, true, false>(in, out, li, op);
    } else {
        if (op.pk >= 0) apply_rc<C64, K, false>(in, out, op);
        else if (op.lctrl >= 0) apply_pair<C64, K, false, true>(in, out, li, op);
        else apply_pair<C64, K, false, false>(in, out, li, op);
    }
}

// Write-back of a group with exit exchanges: register combination r goes to
// the slot of combination x(r) (the affine map of TileGroup), which is one of
// this thread's own slots.
template <bool C64, int K>
__device__ __forceinline__ void write_exit(AmpT<C64> *lds, const Amps<C64, K> &val, uint32_t lbase,
                                           const uint32_t (&soff)[K], CGroup &G)
{
    constexpr int NR = 1 << K;
    uint32_t mb = lbase, ms[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        mb |= ((G.xb >> k) & 1u) ? soff[k] : 0u;
        uint32_t m = 0;
        const uint32_t col = G.xs[k];
#pragma unroll
        for (int k2 = 0; k2 < K; ++k2) m |= ((col >> k2) & 1u) ? soff[k2] : 0u;
        ms[k] = m;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint32_t l = mb;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) l ^= ms[k];
        lds[lds_slot<C64>(l)] = val[r];
    }
}

// Work-group barrier that orders LDS accesses only: global loads issued
// before it may still be in flight after it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A tile amplitude from or to HBM; NT: with the nontemporal hint, for states
// larger than the last-level cache, whose lines a pass touches once.
template <bool NT, typename A>
__device__ __forceinline__ A ld_amp(const A *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename A>
__device__ __forceinline__ void st_amp(A *p, const A &v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Processes tiles g = g0, g0 + gstep, ... below gend of the pass `a` with one
// work-group. Threads tid >= 2^(L-K) (a tile smaller than the work-group) take
// part in the barriers only.
template <bool C64, int K, bool NT = false>
__device__ __forceinline__ void run_tiles(const TileArgs &a, uint64_t g0, uint64_t gend,
                                          uint64_t gstep, AmpT<C64> *lds, AmpT<C64> *tab)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    const uint32_t W = 1u << (a.L - K);
    const uint32_t tid = threadIdx.x;
    const bool active = tid < W;
    A *psi = static_cast<A *>(a.psi);
    CGroup *groups = (CGroup *)(a.groups);
    COp *ops = (COp *)(a.ops);
    const uint64_t *dtab = a.dtab;

    if (a.has_diag) {
        const A *src = static_cast<const A *>(a.phase_tab);
        for (uint32_t i = tid; i < 512; i += blockDim.x) tab[i] = src[i];
    }
    const uint64_t dt = deposit(tid, a.tmask);
    uint64_t roff[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) roff[r] = deposit(uint64_t(r) * W, a.tmask);
    // Relabelled store: output local index lo reads input local index
    // perm(lo), bit j of lo moving to bit osrc_j; perm(tid + r W) =
    // perm(tid) | perm(r W).
    const bool permute = a.permute != 0;
    const uint64_t osrc = a.osrc;
    uint32_t proff[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint32_t x = 0;
        for (int k = 0; k < K; ++k)
            x |= uint32_t((r >> k) & 1) << uint32_t((osrc >> (4 * (a.L - K + k))) & 15u);
        proff[r] = x;
    }

    for (uint64_t g = g0; g < gend; g += gstep) {
        const uint64_t gbase = deposit(g, a.omask);
        // Opaque copies made per tile: the per-slot addresses below are
        // recomputed at each use instead of being hoisted out of the tile loop
        // and held in registers through all the groups.
        uint64_t dtv = dt;
        uint32_t tv = tid;
        asm volatile("" : "+v"(dtv), "+v"(tv));
        if (active) {
            A pv[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) pv[r] = ld_amp<NT>(&psi[gbase | dtv | roff[r]]);
#pragma unroll
            for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(tv + uint32_t(r) * W)] = pv[r];
        }
        // Barriers order LDS accesses only; the tile's global stores of the
        // previous turn may still be in flight.
        lds_barrier();
        for (int gi = 0; gi < a.ngroups; ++gi) {
            CGroup &G = groups[a.group0 + gi];
            // Waves applying a group's ops issue ahead of the other work-group's
            // waves that exchange through LDS or move tiles (layered step
            // -1.8 %, QFT -2.5 % for complex128; -1.7 % / -4.4 % complex64).
            __builtin_amdgcn_s_setprio(2);
            if (active) {
                uint32_t lbase = 0;
                for (int k = 0; k < a.L - K; ++k) lbase |= ((tid >> k) & 1u) << G.ns[k];
                uint32_t soff[K];
#pragma unroll
                for (int k = 0; k < K; ++k) soff[k] = 1u << G.s[k];
                uint32_t li[NR];
                A v[NR], w[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    uint32_t l = lbase;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (r & (1 << k)) l |= soff[k];
                    li[r] = l;
                    v[r] = lds[lds_slot<C64>(l)];
                }
                // Ops alternate v -> w and w -> v; the group ends in either.
                // The write-back applies the group's exit exchanges: only this
                // thread's own slots are permuted, so no barrier is needed.
                const int nops = G.nops;
                const bool exit_map = G.has_exit != 0;
                for (int oi = 0;; oi += 2) {
                    if (oi == nops) {
                        if (exit_map) write_exit<C64, K>(lds, v, lbase, soff, G);
                        else {
#pragma unroll
                            for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(li[r])] = v[r];
                        }
                        break;
                    }
                    apply_op<C64, K>(v, w, li, ops[G.op0 + oi], dtab, a.L, G, g, gbase, tid, tab);
                    if (oi + 1 == nops) {
                        if (exit_map) write_exit<C64, K>(lds, w, lbase, soff, G);
                        else {
#pragma unroll
                            for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(li[r])] = w[r];
                        }
                        break;
                    }
                    apply_op<C64, K>(w, v, li, ops[G.op0 + oi + 1], dtab, a.L, G, g, gbase, tid, tab);
                }
            }
            __builtin_amdgcn_s_setprio(0);
            lds_barrier();
        }
        // Each thread stores the slots it filled, so the next fill needs no
        // barrier, unless the store is relabelled and reads other slots.
        if (active) {
            uint64_t dts = dt;
            uint32_t ts = tid;
            asm volatile("" : "+v"(dts), "+v"(ts));
            const uint64_t gb = gbase | dts;
            if (permute) {
                uint32_t pt = 0;
                for (int j = 0; j < a.L - K; ++j)
                    pt |= ((ts >> j) & 1u) << uint32_t((osrc >> (4 * j)) & 15u);
#pragma unroll
                for (int r = 0; r < NR; ++r) st_amp<NT>(&psi[gb | roff[r]], lds[lds_slot<C64>(pt | proff[r])]);
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) st_amp<NT>(&psi[gb | roff[r]], lds[lds_slot<C64>(ts + uint32_t(r) * W)]);
            }
        }
        if (permute) lds_barrier();
    }
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
    A *tab = lds + (C64 ? size + (size >> 5) : size + (size >> 4));
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
        A *tab = lds + (C64 ? size + (size >> 5) : size + (size >> 4));
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
            A *tab = lds + (C64 ? size + (size >> 5) : size + (size >> 4));
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
