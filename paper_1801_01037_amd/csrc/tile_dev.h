// Device code of the fused tile pass (see kernels_tile.hip): amplitude types,
// the ops applied to a thread's register amplitudes, the register groups'
// LDS exchanges and the walk over a pass's tiles.
//
// The library's generic tile kernel runs a pass's groups and ops from their
// device records in a loop; a pass compiled at run time (jit.hip) runs the
// same functions with every op's kind and register positions fixed at compile
// time. Both include this file, so both apply the same arithmetic; it is also
// built into the library as text for that run-time compilation.
#pragma once

#ifdef __HIPCC_RTC__
#include <type_traits>
#else
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#endif

#include "tile.h"

namespace svk {
namespace dev {

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

// LDS slot of local index l: one padding slot per 32 amplitudes
// (complex64), or one per 16 and one more per 256 (complex128). A 16-byte
// read is served 16 lanes at a time and a write 8 at a time, free of bank
// conflicts when those lanes' slots differ modulo 16 and 8; in the
// complex128 map, local bit b adds 2^(b mod 4) to the slot modulo 16, so
// each register group gives its low thread bits one free tile bit of each
// class b mod 4 (the planner's thread order, TileGroup.ns). The map adds
// over indices with no common bit, lds_slot(a | b) = lds_slot(a) +
// lds_slot(b), since no carry from the low bits can reach a shifted part: a
// thread's slots are its base slot plus offsets that depend on the register
// combination only (constants in a compiled pass).
template <bool C64>
__device__ __forceinline__ uint32_t lds_slot(uint32_t l)
{
    return C64 ? l + (l >> 5) : l + (l >> 4) + (l >> 8);
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

template <typename R>
__device__ __forceinline__ R fmadd(R a, R b, R c)
{
    if constexpr (std::is_same_v<R, float>) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// Complex product with its roundings fixed: in each component one product is
// rounded and the other enters a fused multiply-add. Left to the compiler,
// which product is rounded depends on the surrounding code, and two kernels
// applying the same op could differ in the last bit.
template <typename A>
__device__ __forceinline__ A cmul(A x, A y)
{
    A r;
    r.x = fmadd(x.x, y.x, -(x.y * y.y));
    r.y = fmadd(x.x, y.y, x.y * y.x);
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

// REAL: the matrix has no imaginary parts (a Hadamard); the products with
// its zero parts are left out, which changes no result.
template <bool C64, int K, int PJ, bool SWAP, bool CTRL, bool REAL = false>
__device__ __forceinline__ void pair_pj(const Amps<C64, K> &in, Amps<C64, K> &out, uint32_t lbase,
                                        const uint32_t (&soff)[K], COp &op)
{
    using R = RealT<C64>;
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    // The tile-bit controls: one (lctrl), or several (lcm).
    const uint32_t lm = op.lcm ? op.lcm : (op.lctrl >= 0 ? 1u << op.lctrl : 0u);
    const uint32_t lb = lbase & lm;
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
        } else if constexpr (REAL) {
            na.x = fmadd(m2, b.x, m0 * a.x);
            na.y = fmadd(m2, b.y, m0 * a.y);
            nb.x = fmadd(m6, b.x, m4 * a.x);
            nb.y = fmadd(m6, b.y, m4 * a.y);
        } else {
            na.x = fmadd(-m3, b.y, fmadd(m2, b.x, fmadd(-m1, a.y, m0 * a.x)));
            na.y = fmadd(m3, b.x, fmadd(m2, b.y, fmadd(m1, a.x, m0 * a.y)));
            nb.x = fmadd(-m7, b.y, fmadd(m6, b.x, fmadd(-m5, a.y, m4 * a.x)));
            nb.y = fmadd(m7, b.x, fmadd(m6, b.y, fmadd(m5, a.x, m4 * a.y)));
        }
        if constexpr (CTRL) {
            // the controls of local index lbase | c(r): lbase and c(r)
            // share no bit, so the thread's part is tested once
            uint32_t c = 0;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (r & (1 << k)) c |= soff[k];
            const bool on = (lb | (c & lm)) == lm;
            out[r] = on ? na : a;
            out[r1] = on ? nb : b;
        } else {
            out[r] = na;
            out[r1] = nb;
        }
    }
}

template <bool C64, int K, bool SWAP, bool CTRL>
__device__ __forceinline__ void apply_pair(const Amps<C64, K> &in, Amps<C64, K> &out, uint32_t lbase,
                                           const uint32_t (&soff)[K], COp &op)
{
    // The planner emits positions below K only; the other arms are unreachable
    // (an arm that wrote nothing, or copied, would keep the other array live or
    // be hoisted in front of every op).
    switch (op.pj) {
    case 0: pair_pj<C64, K, 0, SWAP, CTRL>(in, out, lbase, soff, op); break;
    case 1:
        if constexpr (K > 1) pair_pj<C64, K, 1, SWAP, CTRL>(in, out, lbase, soff, op);
        else __builtin_unreachable();
        break;
    case 2:
        if constexpr (K > 2) pair_pj<C64, K, 2, SWAP, CTRL>(in, out, lbase, soff, op);
        else __builtin_unreachable();
        break;
    case 3:
        if constexpr (K > 3) pair_pj<C64, K, 3, SWAP, CTRL>(in, out, lbase, soff, op);
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

// The turns of a diagonal op (the quadratic phase form described with
// TileOp) for this thread and tile: base, and coef_k for the register
// positions k in LIN. Positions outside LIN are left zero, and so is base
// unless BASE: callers pass only what the op's shape (TileOp.dlin) allows to
// be non-zero.
template <int K, uint32_t LIN, bool BASE>
__device__ __forceinline__ void diag_turns(COp &op, const uint64_t *dtab, int L, CGroup &G,
                                           uint64_t g, uint32_t tid, uint64_t &base,
                                           uint64_t (&coef)[K])
{
    const uint64_t *th = dtab + op.dthr + size_t(tid) * (K + 1);
    base = BASE ? th[0] : 0;
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = ((LIN >> k) & 1u) ? th[1 + k] : 0;
    if (op.dout >= 0) {
        // Weights against the bits of g: uniform byte-table sums (scalar loads).
        CU64 *bt = (CU64 *)(dtab + op.dout);
        auto ow = [&](int l) {
            uint64_t w = 0;
            for (int b = 0; b < op.dbytes; ++b)
                w += bt[(size_t(b) * (L + 1) + l) * 256 + ((g >> (8 * b)) & 255u)];
            return w;
        };
        if constexpr (BASE) {
            base += ow(L);
            for (int k = 0; k < L - K; ++k) {
                const uint64_t w = ow(G.ns[k]);
                base += ((tid >> k) & 1u) ? w : 0ull;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((LIN >> k) & 1u) coef[k] += ow(G.s[k]);
    }
}

// Diagonal op: the turn of register combination r is base + sum_{k in r}
// coef_k + PR(r), so the phase of every amplitude is a product of five
// evaluated phases and a constant.
template <bool C64, int K>
__device__ __forceinline__ void apply_diag(const Amps<C64, K> &in, Amps<C64, K> &out, COp &op,
                                           const uint64_t *dtab, int L, CGroup &G, uint64_t g,
                                           uint32_t tid, const AmpT<C64> *tab)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    uint64_t base, coef[K];
    diag_turns<K, (1u << K) - 1, true>(op, dtab, L, G, g, tid, base, coef);
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

// The same op with its shape fixed at compile time: LIN and BASE as in
// TileOp.dlin, and ONE the register combinations whose constant factor
// e^{2 pi i PR(r) / 2^64} is exactly 1. Phases that are exactly 1 are neither
// evaluated nor multiplied (a controlled phase on a register pivot changes
// only the half of the amplitudes with the pivot set); the factors that
// remain are multiplied in the generic op's order, so the results are the
// same.
template <bool C64, int K, uint32_t LIN, bool BASE, uint32_t ONE>
__device__ __forceinline__ void apply_diag_shape(const Amps<C64, K> &in, Amps<C64, K> &out,
                                                 COp &op, const uint64_t *dtab, int L, CGroup &G,
                                                 uint64_t g, uint32_t tid, const AmpT<C64> *tab)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    uint64_t base, coef[K];
    diag_turns<K, LIN, BASE>(op, dtab, L, G, g, tid, base, coef);
    A ek[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        if ((LIN >> k) & 1u) ek[k] = turn_phase<C64>(coef[k], tab);
    // p[r]: the product of r's evaluated phases (set only where it is not 1).
    A p[NR];
    if constexpr (BASE) p[0] = turn_phase<C64>(base, tab);
#pragma unroll
    for (int r = 1; r < NR; ++r) {
        const uint32_t rl = uint32_t(r) & LIN;
        if (rl == 0) {
            if (BASE) p[r] = p[0];
            continue;
        }
        const int k = 31 - __builtin_clz(rl);
        const int prev = r ^ (1 << k);
        p[r] = (!BASE && (uint32_t(prev) & LIN) == 0) ? ek[k] : cmul(p[prev], ek[k]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const bool one_p = !BASE && (uint32_t(r) & LIN) == 0;
        const bool one_c = (ONE >> r) & 1u;
        if (one_p && one_c) {
            out[r] = in[r];
            continue;
        }
        A c{};
        if (!one_c) {
            if constexpr (C64) { c.x = op.mf4[2 * r]; c.y = op.mf4[2 * r + 1]; }
            else { c.x = op.m4[2 * r]; c.y = op.m4[2 * r + 1]; }
        }
        const A f = one_p ? c : (one_c ? p[r] : cmul(p[r], c));
        out[r] = cmul(in[r], f);
    }
}

// Applies one op of group G: in -> out.
template <bool C64, int K>
__device__ __forceinline__ void apply_op(const Amps<C64, K> &in, Amps<C64, K> &out,
                                         uint32_t lbase, const uint32_t (&soff)[K], COp &op,
                                         const uint64_t *dtab, int L, CGroup &G, uint64_t g,
                                         uint64_t gbase, uint32_t tid, const AmpT<C64> *tab)
{
    if (op.kind == TOP_DIAG) {
        apply_diag<C64, K>(in, out, op, dtab, L, G, g, tid, tab);
    } else if (op.kind == TOP_U4) {
        apply_u4<C64, K>(in, out, op);
    } else if ((op.octrl >= 0 && !((gbase >> op.octrl) & 1ull)) ||
               (op.ocm && (gbase & op.ocm) != op.ocm)) {
        copy_amps<C64, K>(in, out);   // a control outside the tile is 0 here
    } else if (op.kind == TOP_SWAP) {
        if (op.pk >= 0) apply_rc<C64, K, true>(in, out, op);
        else if (op.lctrl >= 0 || op.lcm) apply_pair<C64, K, true, true>(in, out, lbase, soff, op);
        else apply_pair<C64, K, true, false>(in, out, lbase, soff, op);
    } else {
        if (op.pk >= 0) apply_rc<C64, K, false>(in, out, op);
        else if (op.lctrl >= 0 || op.lcm) apply_pair<C64, K, false, true>(in, out, lbase, soff, op);
        else apply_pair<C64, K, false, false>(in, out, lbase, soff, op);
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

// The same with the map given as a table, for register bits fixed at
// compile time (a compiled pass): the thread's base slot plus a constant
// offset per register.
template <bool C64, int K>
__device__ __forceinline__ void write_map(AmpT<C64> *lds, const Amps<C64, K> &val, uint32_t lbase,
                                          const uint32_t (&soff)[K], const uint32_t (&xr)[1 << K])
{
    uint32_t sb = lds_slot<C64>(lbase);
    asm volatile("" : "+v"(sb));
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) c |= ((xr[r] >> k) & 1u) ? soff[k] : 0u;
        lds[sb + lds_slot<C64>(c)] = val[r];
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

// Index bit of the s-th set bit of mask (mask uniform, s a constant).
__device__ __forceinline__ uint64_t nth_bit(uint64_t mask, int s)
{
    for (int i = 0; i < s; ++i) mask &= mask - 1;
    return mask & (~mask + 1);
}

// Direct transfers between HBM and a group's registers, with no LDS round
// trip: a pass's first group can take its amplitudes fetched from HBM in its
// own layout and its last group can store them there, when the threads' own
// bits keep the tile's low index bits (coalesced accesses). rb[k] is the
// index bit of register bit k; gb holds the tile's outside bits and the
// thread's own bits.
template <bool C64, int K, bool NT>
__device__ __forceinline__ void fetch_direct(const TileArgs &a, uint64_t gb, const uint64_t (&rb)[K],
                                             Amps<C64, K> &v)
{
    using A = AmpT<C64>;
    const A *psi = static_cast<const A *>(a.psi);
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint64_t x = gb;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) x |= rb[k];
        v[r] = ld_amp<NT>(&psi[x]);
    }
}

// A group's registers taken from amplitudes fetched in its own layout.
template <bool C64, int K>
__device__ __forceinline__ void take_regs(const Amps<C64, K> &cur, Amps<C64, K> &v)
{
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) v[r] = cur[r];
}

// Register combination r goes to the index of combination xr[r] (the group's
// exit map, or r itself); ob[k] is the index bit that register bit k is
// written to (the pass's relabelled order when it has one).
template <bool C64, int K, bool NT>
__device__ __forceinline__ void store_direct(const TileArgs &a, uint64_t gb, const uint64_t (&ob)[K],
                                             const uint32_t (&xr)[1 << K], const Amps<C64, K> &v)
{
    using A = AmpT<C64>;
    A *psi = static_cast<A *>(a.psi);
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint64_t x = gb;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (xr[r] & (1u << k)) x |= ob[k];
        st_amp<NT>(&psi[x], v[r]);
    }
}

// Per-thread constants of one pass's walk over its tiles. Register r's
// offsets are linear in the bits of r, so only the K basis values are kept;
// each use rebuilds r's offset from them (scalar ORs) instead of holding all
// 2^K offsets in scalar registers through the tile loop.
template <int K>
struct Walk {
    uint32_t W;            // threads holding amplitudes: 2^(L-K)
    uint32_t tid;
    bool active;           // tid < W (a tile smaller than the work-group)
    uint64_t dt;           // this thread's tile bits as index bits
    uint64_t rbit[K];      // index bit of register bit k
    uint32_t pbit[K];      // local bit that register bit k reads under the relabelled store
};

// Offset of register combination r from per-bit basis values b (each a
// single bit): their OR over the set bits of r. The basis is copied through
// an opaque move first, so the 2^K combinations are formed where they are
// used rather than hoisted out of the tile loop.
template <int K, typename T>
__device__ __forceinline__ void reg_offsets(const T (&b)[K], T (&out)[1 << K])
{
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = b[k];
        asm volatile("" : "+s"(v[k]));
    }
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        T x = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) x |= v[k];
        out[r] = x;
    }
}

// Loads the phase table (passes with diagonal ops) and the walk constants.
template <bool C64, int K>
__device__ __forceinline__ void walk_init(const TileArgs &a, AmpT<C64> *tab, Walk<K> &w)
{
    using A = AmpT<C64>;
    w.W = 1u << (a.L - K);
    w.tid = threadIdx.x;
    w.active = w.tid < w.W;
    if (a.has_diag) {
        const A *src = static_cast<const A *>(a.phase_tab);
        for (uint32_t i = w.tid; i < 512; i += blockDim.x) tab[i] = src[i];
    }
    w.dt = deposit(w.tid, a.tmask);
#pragma unroll
    for (int k = 0; k < K; ++k) w.rbit[k] = nth_bit(a.tmask, a.L - K + k);
    // Relabelled store: output local index lo reads input local index
    // perm(lo), bit j of lo moving to bit osrc_j; perm(tid + r W) =
    // perm(tid) | perm(r W).
#pragma unroll
    for (int k = 0; k < K; ++k) w.pbit[k] = 1u << uint32_t((a.osrc >> (4 * (a.L - K + k))) & 15u);
}

// Tile g (index bits outside the tile = gbase) from HBM into LDS, then a
// barrier that orders LDS only (the previous tile's global stores may still
// be in flight). WAIT: the previous tile ended in direct stores, whose last
// group read other threads' slots, so the slots are written only after a
// barrier.
template <bool C64, int K, bool NT, bool WAIT = false>
__device__ __forceinline__ void tile_load(const TileArgs &a, const Walk<K> &w, uint64_t gbase,
                                          AmpT<C64> *lds)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    const A *psi = static_cast<const A *>(a.psi);
    // Opaque copies made per tile: the per-slot addresses below are
    // recomputed at each use instead of being hoisted out of the tile loop
    // and held in registers through all the groups.
    uint64_t dtv = w.dt;
    uint32_t tv = w.tid;
    asm volatile("" : "+v"(dtv), "+v"(tv));
    A pv[NR];
    if (w.active) {
        uint64_t roff[NR];
        reg_offsets<K>(w.rbit, roff);
#pragma unroll
        for (int r = 0; r < NR; ++r) pv[r] = ld_amp<NT>(&psi[gbase | dtv | roff[r]]);
    }
    if constexpr (WAIT) lds_barrier();
    if (w.active) {
#pragma unroll
        for (int r = 0; r < NR; ++r) lds[lds_slot<C64>(tv) + lds_slot<C64>(uint32_t(r) * w.W)] = pv[r];
    }
    lds_barrier();
}

// The fetch of walks whose first group does not take fetched registers.
struct NoFetch {
    template <typename W, typename R>
    __device__ __forceinline__ void operator()(uint64_t, const W &, R &) const {}
};

// The tile from LDS back to HBM, in the relabelled order when the pass has
// one. Each thread stores the slots it filled, so the next fill needs no
// barrier, unless the store is relabelled and reads other slots.
template <bool C64, int K, bool NT>
__device__ __forceinline__ void tile_store(const TileArgs &a, const Walk<K> &w, uint64_t gbase,
                                           const AmpT<C64> *lds)
{
    using A = AmpT<C64>;
    constexpr int NR = 1 << K;
    A *psi = static_cast<A *>(a.psi);
    const bool permute = a.permute != 0;
    if (w.active) {
        uint64_t dts = w.dt;
        uint32_t ts = w.tid;
        asm volatile("" : "+v"(dts), "+v"(ts));
        const uint64_t gb = gbase | dts;
        uint64_t roff[NR];
        reg_offsets<K>(w.rbit, roff);
        if (permute) {
            uint32_t pt = 0;
            for (int j = 0; j < a.L - K; ++j)
                pt |= ((ts >> j) & 1u) << uint32_t((a.osrc >> (4 * j)) & 15u);
            uint32_t proff[NR];
            reg_offsets<K>(w.pbit, proff);
#pragma unroll
            for (int r = 0; r < NR; ++r)
                st_amp<NT>(&psi[gb | roff[r]], lds[lds_slot<C64>(pt) + lds_slot<C64>(proff[r])]);
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                st_amp<NT>(&psi[gb | roff[r]], lds[lds_slot<C64>(ts) + lds_slot<C64>(uint32_t(r) * w.W)]);
        }
    }
    if (permute) lds_barrier();
}

// A group's register amplitudes: register combination r holds local index
// lbase | c(r), the thread's fixed tile bits lbase plus the set bits of r
// placed at the group's register bits (soff[k] = 1 << s_k), read from LDS.
// Register bits known only at run time (the generic kernel): each slot is
// computed from its full local index.
template <bool C64, int K>
__device__ __forceinline__ void gather(const AmpT<C64> *lds, uint32_t lbase,
                                       const uint32_t (&soff)[K], Amps<C64, K> &v)
{
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) c |= soff[k];
        v[r] = lds[lds_slot<C64>(lbase | c)];
    }
}

// A group's write-back: to the slots it read, or through its exit map.
template <bool C64, int K>
__device__ __forceinline__ void scatter(AmpT<C64> *lds, const Amps<C64, K> &v, uint32_t lbase,
                                        const uint32_t (&soff)[K], CGroup &G, bool exit_map)
{
    if (exit_map) {
        write_exit<C64, K>(lds, v, lbase, soff, G);
    } else {
#pragma unroll
        for (int r = 0; r < (1 << K); ++r) {
            uint32_t c = 0;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (r & (1 << k)) c |= soff[k];
            lds[lds_slot<C64>(lbase | c)] = v[r];
        }
    }
}

// The same two for register bits fixed at compile time (a compiled pass):
// the thread's base slot plus a constant offset per register, which the
// LDS instructions take as immediates.
template <bool C64, int K>
__device__ __forceinline__ void gather_fixed(const AmpT<C64> *lds, uint32_t lbase,
                                             const uint32_t (&soff)[K], Amps<C64, K> &v)
{
    const uint32_t sb = lds_slot<C64>(lbase);
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) c |= soff[k];
        v[r] = lds[sb + lds_slot<C64>(c)];
    }
}

template <bool C64, int K>
__device__ __forceinline__ void scatter_fixed(AmpT<C64> *lds, const Amps<C64, K> &v, uint32_t lbase,
                                              const uint32_t (&soff)[K])
{
    // An opaque base: the slots are recomputed here instead of being
    // carried in registers from the gather through all the ops.
    uint32_t sb = lds_slot<C64>(lbase);
    asm volatile("" : "+v"(sb));
#pragma unroll
    for (int r = 0; r < (1 << K); ++r) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (r & (1 << k)) c |= soff[k];
        lds[sb + lds_slot<C64>(c)] = v[r];
    }
}

// Processes tiles g = g0, g0 + gstep, ... below gend of the pass `a` with one
// work-group: each tile is loaded into LDS (with DF instead fetched into
// registers by `fetch`, in the first group's own layout), `groups(g, gbase,
// w, regs)` runs the pass's register groups on it (every group ending in a
// work-group barrier; with DF the first group takes the fetched registers),
// and it is stored (unless DL: the last group stores it and ends without a
// barrier). Threads tid >= 2^(L-K) (a tile smaller than the work-group) take
// part in the barriers only.
template <bool C64, int K, bool NT, bool DF = false, bool DL = false, typename Groups,
          typename Fetch>
__device__ __forceinline__ void walk_tiles(const TileArgs &a, uint64_t g0, uint64_t gend,
                                           uint64_t gstep, AmpT<C64> *lds, AmpT<C64> *tab,
                                           const Groups &groups, const Fetch &fetch)
{
    Walk<K> w;
    walk_init<C64, K>(a, tab, w);
    // A first group that takes fetched registers runs its ops before any
    // barrier: the phase table must be in LDS before.
    if constexpr (DF) lds_barrier();
    for (uint64_t g = g0; g < gend; g += gstep) {
        const uint64_t gbase = deposit(g, a.omask);
        // Only a DF walk fills these registers; loading through them in the
        // other walks would hold them live and costs the generic kernels
        // their registers.
        Amps<C64, K> cur;
        if constexpr (DF) fetch(gbase, w, cur);
        else tile_load<C64, K, NT, DL>(a, w, gbase, lds);
        groups(g, gbase, w, cur);
        if constexpr (!DL) tile_store<C64, K, NT>(a, w, gbase, lds);
    }
}

}  // namespace dev
}  // namespace svk
