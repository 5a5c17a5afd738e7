// Circuit planning for SV_FUSE: gate list -> tile passes.
//
// The paper applies one gate per sweep over the state (Algorithm 1). On one
// GPU every sweep is bound by HBM, so the planner packs as many gates as it
// legally can into one sweep:
//   * a pass owns a set T of L tile qubits (index bits 0..nlow-1 always, for
//     coalesced access, plus the targets met first in the gate list);
//   * a non-diagonal gate joins the pass when its target is in T and it does
//     not touch a qubit of a gate already left for a later pass (gates on
//     disjoint qubits commute, so skipping ahead over them is exact);
//   * a diagonal gate (controlled phase, or diag(1, e^{i phi})) joins any
//     pass, and is held back inside the pass until the first later op that
//     touches one of its qubits: diagonal gates commute with each other and
//     with everything on other qubits, so held-back phases merge into few
//     diagonal ops. Phases are kept as exact uint64 fractions of a turn;
//   * inside a pass, consecutive ops whose targets fit in K register bits form
//     a group (one LDS exchange per group); runs of gates on two qubits are
//     multiplied into 4x4 ops, and exchanges that end a group ride on its
//     write-back. Two ways of forming the blocks are tried per pass and the
//     one with the lower estimated cost is kept;
//   * between passes the qubits may be relabelled (section Non-Sequential
//     Storage of the State Vector): a pass writes its tile back with the
//     qubits the next gates need in the index bits every tile must hold.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "dense.h"
#include "plan.h"
#include "tile.h"

namespace svk {
namespace {

// One gate after classification.
struct Item {
    int gate = -1;
    bool diag = false;
    int target = -1, control = -1;   // non-diagonal
    uint64_t xcm = 0;                // further controls (several-control gates)
    bool swap = false;
    double m[8] = {};
    int pivot = -1, wbit = -1;       // diagonal: pivot bit, weight bit (-1: constant)
    uint64_t turn = 0;
    uint64_t qmask = 0;              // qubits touched
};

// A diagonal term: e^{2 pi i turn / 2^64} where bit p is 1 and (wbit < 0 or
// bit wbit is 1).
struct DTerm {
    int wbit;
    uint64_t turn;
    int gate;
};

struct PPivot {
    int p = -1;
    std::vector<DTerm> terms;
};

struct POp {
    int kind = TOP_U;
    int target = -1, control = -1;
    uint64_t xcm = 0;          // TOP_U / TOP_SWAP: controls besides `control`
    double m[8] = {};
    std::vector<PPivot> piv;
    std::vector<int> gates;
    int q0 = -1, q1 = -1;      // TOP_U4: its two qubits, q0 < q1
    double m4[32] = {};        // TOP_U4: 4x4, basis b0 + 2 b1 (b0 = bit q0, b1 = bit q1)
};

// Qubits an op touches (a diagonal op: its pivots and weight bits).
uint64_t op_qmask(const POp &op)
{
    if (op.kind == TOP_U4) return (uint64_t(1) << op.q0) | (uint64_t(1) << op.q1);
    if (op.kind != TOP_DIAG)
        return (uint64_t(1) << op.target) | (op.control >= 0 ? uint64_t(1) << op.control : 0) |
               op.xcm;
    uint64_t m = 0;
    for (const PPivot &P : op.piv) {
        m |= uint64_t(1) << P.p;
        for (const DTerm &t : P.terms)
            if (t.wbit >= 0) m |= uint64_t(1) << t.wbit;
    }
    return m;
}

// Applies a 2x2 (optionally controlled) op to the 4 columns of a 4x4 matrix
// over qubits (q0, q1); column-major work on (re, im) pairs.
void apply_to_4x4(const POp &op, int q0, double *mat /* 4x4 complex, row major */)
{
    const int t = op.target == q0 ? 0 : 1;
    const int c = op.control < 0 ? -1 : (op.control == q0 ? 0 : 1);
    double g[8];
    if (op.kind == TOP_SWAP) {
        const double x[8] = {0, 0, 1, 0, 1, 0, 0, 0};
        std::memcpy(g, x, sizeof g);
    } else {
        std::memcpy(g, op.m, sizeof g);
    }
    for (int col = 0; col < 4; ++col)
        for (int i0 = 0; i0 < 4; ++i0) {
            if ((i0 >> t) & 1) continue;
            if (c >= 0 && !((i0 >> c) & 1)) continue;
            const int i1 = i0 | (1 << t);
            double *a = mat + (i0 * 4 + col) * 2, *b = mat + (i1 * 4 + col) * 2;
            const double ar = a[0], ai = a[1], br = b[0], bi = b[1];
            a[0] = g[0] * ar - g[1] * ai + g[2] * br - g[3] * bi;
            a[1] = g[0] * ai + g[1] * ar + g[2] * bi + g[3] * br;
            b[0] = g[4] * ar - g[5] * ai + g[6] * br - g[7] * bi;
            b[1] = g[4] * ai + g[5] * ar + g[6] * bi + g[7] * br;
        }
}

// Inside one register group, merges runs of ops that act on at most two
// register qubits into one op: a 4x4 over the two qubits, or a product 2x2 on
// one. Ops are taken in the light-cone order of the pass planner: an op may
// move ahead of ops it shares no qubit with. Ops with a control outside the
// register qubits, and diagonal ops, are kept as they are. A run of a single op
// is kept too (an exchange or a 2x2 is cheaper than a 4x4).
// Estimated cost of one op in a tile pass, in FP64 operations per amplitude:
// its arithmetic plus a fixed part (reading the op record, one pass of the
// register amplitudes from one array to the other). Fitted to measured
// passes: a 4x4 costs about 3.3 times an exchange and 1.6 times a 2x2.
double op_cost(const POp &op)
{
    switch (op.kind) {
    case TOP_U4: return 43.0;
    case TOP_U: return 27.0;
    case TOP_SWAP: return 13.0;
    default: return 25.0;   // TOP_DIAG
    }
}
constexpr double kGroupCost = 25.0;   // one LDS exchange of the register amplitudes
constexpr int kCoverMinQubits = 26;    // states that get the coverage search for groups
constexpr int kCoverPool = 8;          // qubits its candidate register sets are drawn from
constexpr double kPassFloor = 415.0;  // a pass's HBM time on the same scale

// spread = false: each block is seeded with the first two-qubit op left;
// spread = true: a two-qubit op that reaches the front of the list stays
// alone, and a block is seeded with the first two-qubit op on the front op's
// qubit. On layered circuits the second lets one 4x4 take two layers of
// one-qubit gates around every other layer of CNOTs, which stay exchanges.
std::vector<POp> fuse_group(std::vector<POp> ops, uint64_t regq, bool spread)
{
    auto absorbable = [&](const POp &op) {
        if ((op.kind != TOP_U && op.kind != TOP_SWAP) || op.xcm) return false;
        return op.control < 0 || ((regq >> op.control) & 1);
    };
    std::vector<uint64_t> qmask(ops.size());
    uint64_t all_q = 0;   // every qubit the ops touch
    for (size_t i = 0; i < ops.size(); ++i) all_q |= qmask[i] = op_qmask(ops[i]);
    auto is2q = [&](int i) { return __builtin_popcountll(qmask[i]) == 2; };
    std::vector<POp> out;
    out.reserve(ops.size());
    std::vector<int> live(ops.size()), members, next;
    for (size_t i = 0; i < ops.size(); ++i) live[i] = int(i);
    size_t head = 0;   // live[head..] are the ops still to place, in order
    while (head < live.size()) {
        const int f = live[head];
        // With `spread`, a two-qubit op with no op left before it stays alone:
        // the one-qubit ops that follow it can join the next block on their
        // qubits, and a block seeded here would cost a 4x4 for what an
        // exchange or a controlled 2x2 does.
        if (!absorbable(ops[f]) || (spread && is2q(f))) {
            out.push_back(std::move(ops[f]));
            ++head;
            continue;
        }
        // Seed the block with the qubits of a two-qubit op, so that it
        // collects the one-qubit ops before and after that gate.
        uint64_t seed = qmask[f];
        for (size_t k = head; k < live.size(); ++k) {
            const int i = live[k];
            if (absorbable(ops[i]) && is2q(i) && (!spread || (qmask[i] & seed))) {
                seed = qmask[i];
                break;
            }
        }
        members.clear();
        for (int attempt = 0; attempt < 2 && members.empty(); ++attempt) {
            if (attempt == 1) seed = qmask[f];   // the seed could not join
            uint64_t P = seed, blocked = 0;
            next.clear();
            for (size_t k = head; k < live.size(); ++k) {
                const int i = live[k];
                const uint64_t qm = qmask[i];
                if ((blocked & all_q) == all_q) {   // nothing later can join
                    next.insert(next.end(), live.begin() + long(k), live.end());
                    break;
                }
                if ((qm & blocked) || !absorbable(ops[i]) || __builtin_popcountll(P | qm) > 2) {
                    blocked |= qm;
                    next.push_back(i);
                    continue;
                }
                P |= qm;
                members.push_back(i);
            }
        }
        uint64_t P = 0;
        double alone = 0;   // cost of the members as they are
        for (int i : members) {
            P |= qmask[i];
            alone += op_cost(ops[i]);
        }
        POp probe;
        probe.kind = TOP_U4;
        if (members.size() == 1 || (__builtin_popcountll(P) == 2 && alone <= op_cost(probe))) {
            // a 4x4 would not be cheaper
            for (int i : members) out.push_back(std::move(ops[i]));
        } else if (__builtin_popcountll(P) == 1) {
            // product of 2x2s on one qubit (each later op multiplies on the left)
            POp fo;
            fo.kind = TOP_U;
            fo.target = ops[members.front()].target;
            double acc[8] = {1, 0, 0, 0, 0, 0, 1, 0};
            for (int i : members) {
                const POp &mop = ops[i];
                double g[8];
                if (mop.kind == TOP_SWAP) {
                    const double x[8] = {0, 0, 1, 0, 1, 0, 0, 0};
                    std::memcpy(g, x, sizeof g);
                } else {
                    std::memcpy(g, mop.m, sizeof g);
                }
                double r[8];
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        double re = 0, im = 0;
                        for (int k = 0; k < 2; ++k) {
                            const double gr = g[(2 * a + k) * 2], gi = g[(2 * a + k) * 2 + 1];
                            const double ar = acc[(2 * k + b) * 2], ai = acc[(2 * k + b) * 2 + 1];
                            re += gr * ar - gi * ai;
                            im += gr * ai + gi * ar;
                        }
                        r[(2 * a + b) * 2] = re;
                        r[(2 * a + b) * 2 + 1] = im;
                    }
                std::memcpy(acc, r, sizeof acc);
                fo.gates.insert(fo.gates.end(), mop.gates.begin(), mop.gates.end());
            }
            std::memcpy(fo.m, acc, sizeof acc);
            out.push_back(std::move(fo));
        } else {
            POp fo;
            fo.kind = TOP_U4;
            fo.q0 = __builtin_ctzll(P);
            fo.q1 = 63 - __builtin_clzll(P);
            for (int k = 0; k < 4; ++k) fo.m4[(k * 4 + k) * 2] = 1.0;
            for (int i : members) {
                apply_to_4x4(ops[i], fo.q0, fo.m4);
                fo.gates.insert(fo.gates.end(), ops[i].gates.begin(), ops[i].gates.end());
            }
            out.push_back(std::move(fo));
        }
        live.swap(next);
        head = 0;
    }
    return out;
}

struct PGroup {
    std::vector<int> S;   // local positions
    std::vector<POp> ops;
    std::vector<POp> folded;   // exchanges applied by the write-back (TileGroup exit map)
    uint32_t xb = 0;
    uint32_t xs[kTileMaxK] = {1, 2, 4, 8};
};

// Moves the exchanges (X, CNOT) on register qubits that no later op of the
// group touches out of the op list into the group's exit map: they commute
// with every later op, so they can be applied last, as a permutation of each
// thread's register combinations when the group writes back to LDS.
void fold_exit(PGroup &g, const std::vector<int> &T)
{
    uint64_t regq = 0;   // storage bits of the register positions
    for (int sidx : g.S) regq |= uint64_t(1) << T[sidx];
    auto rpos = [&](int b) {
        for (int k = 0; k < int(g.S.size()); ++k)
            if (T[g.S[k]] == b) return k;
        return -1;
    };
    uint64_t kept = 0;
    std::vector<char> out(g.ops.size(), 0);
    bool any = false;
    for (int i = int(g.ops.size()) - 1; i >= 0; --i) {
        const POp &op = g.ops[i];
        const uint64_t qm = op_qmask(op);
        const bool exch = op.kind == TOP_SWAP && !op.xcm && ((regq >> op.target) & 1) &&
                          (op.control < 0 || ((regq >> op.control) & 1));
        if (exch && !(qm & kept)) {
            out[i] = 1;
            any = true;
        } else {
            kept |= qm;
        }
    }
    if (!any) return;
    std::vector<POp> keep, fold;
    for (size_t i = 0; i < g.ops.size(); ++i) (out[i] ? fold : keep).push_back(std::move(g.ops[i]));
    // x = E_m ... E_1 (r): an X on position t adds e_t, a CNOT c -> t adds
    // bit c to bit t; composed in gate order on the columns and the constant.
    for (const POp &op : fold) {
        const int t = rpos(op.target);
        if (op.control < 0) {
            g.xb ^= 1u << t;
            continue;
        }
        const int c = rpos(op.control);
        for (int k = 0; k < kTileMaxK; ++k) g.xs[k] ^= ((g.xs[k] >> c) & 1u) << t;
        g.xb ^= ((g.xb >> c) & 1u) << t;
    }
    g.ops = std::move(keep);
    g.folded = std::move(fold);
}

struct PPass {
    std::vector<int> T;   // index bits of the tile (storage positions), ascending
    std::vector<PGroup> groups;
    std::vector<int> osrc;   // output local bit j takes input local bit osrc[j]
                             // (empty: the tile is written back in its own order)
};

// Storage order of the qubits between passes (the paper's non-sequential
// storage of the state vector): logical qubit q is stored at index bit
// pos[q]; inv is the inverse. A pass may permute the qubits of its own tile
// on the way out, so its tile still covers the same amplitudes and it stays
// in place.
struct Layout {
    std::vector<int> pos, inv;
    explicit Layout(int n) : pos(n), inv(n)
    {
        for (int q = 0; q < n; ++q) pos[q] = inv[q] = q;
    }
    bool identity() const
    {
        for (size_t q = 0; q < pos.size(); ++q)
            if (pos[q] != int(q)) return false;
        return true;
    }
};

// Rewrites an op's qubits as storage positions.
void to_storage(POp &op, const std::vector<int> &pos)
{
    if (op.target >= 0) op.target = pos[op.target];
    if (op.control >= 0) op.control = pos[op.control];
    uint64_t x = 0;
    for (uint64_t m = op.xcm; m; m &= m - 1) x |= uint64_t(1) << pos[__builtin_ctzll(m)];
    op.xcm = x;
    for (PPivot &P : op.piv) {
        P.p = pos[P.p];
        for (DTerm &t : P.terms)
            if (t.wbit >= 0) t.wbit = pos[t.wbit];
    }
}

// Qubits in the order a restoring pass wants them: each cycle of the storage
// permutation walked from a qubit held in the low index bits (q, then the
// qubit whose home q occupies, ...), then the other cycles. A tile holding a
// run of a cycle sends every member but the first home.
std::vector<int> cycle_order(const Layout &lay, int nlow)
{
    const int n = int(lay.pos.size());
    std::vector<char> seen(n, 0);
    std::vector<int> out;
    auto walk = [&](int start) {
        int q = start;
        while (!seen[q]) {
            seen[q] = 1;
            out.push_back(q);
            q = lay.pos[q];
        }
    };
    for (int b = 0; b < nlow && b < n; ++b)
        if (lay.inv[b] != b) walk(lay.inv[b]);
    for (int q = 0; q < n; ++q)
        if (lay.pos[q] != q) walk(q);
    return out;
}

struct TileGeom {
    int L, K, nlow;
    bool fuse4;     // merge register-local runs into 4x4 ops
    bool c64;
    bool nlow_free; // nlow is the default, not set by the environment or the handle
};

// Fixed low tile qubits of the second plan tried for states past the
// last-level cache: contiguous runs of 1 KiB (complex128) or 512 B (complex64).
constexpr int kLongRunLow = 6;

// The tile geometry of a state; `s` (optional) carries the overrides set by
// sv_set_tile_geometry, applied after the environment's tuning overrides.
TileGeom geometry(int n, sv_dtype dt, int force_k = 0, const sv_state_s *s = nullptr)
{
    const bool c64 = dt == SV_C64;
    TileGeom g;
    g.c64 = c64;
    int L = c64 ? kTileL64 : kTileL128;
    int K = c64 ? kTileK64 : kTileK128;
    // Fixed low tile qubits: contiguous runs of one 128 B line, so no line is
    // shared by two tiles (and fetched twice).
    int nlow = c64 ? 4 : 3;
    // Tuning overrides (bounded to what the kernels are built for).
    if (const char *e = std::getenv("SV_TILE_L")) L = std::max(4, std::min(std::atoi(e), L));
    if (const char *e = std::getenv("SV_TILE_K")) K = std::max(3, std::min(std::atoi(e), 4));
    g.nlow_free = true;
    if (const char *e = std::getenv("SV_TILE_NLOW")) {
        nlow = std::atoi(e);
        g.nlow_free = false;
    }
    if (s) {
        if (s->tile_L > 0) L = std::min(s->tile_L, L);
        if (s->tile_K > 0) K = s->tile_K;
        if (s->tile_nlow >= 0) {
            nlow = s->tile_nlow;
            g.nlow_free = false;
        }
    }
    g.fuse4 = true;
    if (const char *e = std::getenv("SV_TILE_FUSE4")) g.fuse4 = std::atoi(e) != 0;
    if (force_k > 0) K = force_k;
    g.L = std::min(n, L);
    g.K = std::min(g.L, K);
    if (g.L - g.K > 10) g.K = g.L - 10;   // at most 1024 threads
    // At least one tile bit must stay free for other targets when the tile
    // does not cover the whole register, or no pass could admit them.
    g.nlow = std::max(0, std::min(nlow, g.L < n ? g.L - 1 : g.L));
    return g;
}

Item classify(const sv_gate &g, int idx)
{
    Item it;
    it.gate = idx;
    const uint64_t tb = uint64_t(1) << g.target;
    if (g.kind == SV_G_MCU) {
        // Several controls: the lowest is `control`, the others go with it
        // as a mask; never a diagonal term (those hold at most two qubits).
        const uint64_t cm = uint64_t(uint32_t(g.control)) | (uint64_t(uint32_t(g.flags)) << 32);
        it.target = g.target;
        it.control = __builtin_ctzll(cm);
        it.xcm = cm & (cm - 1);
        it.swap = is_pauli_x(g.m);
        std::memcpy(it.m, g.m, sizeof it.m);
        it.qmask = tb | cm;
        return it;
    }
    if (g.kind == SV_G_CPHASE || (g.kind != SV_G_U && is_phase_diag(g.m)) ||
        (g.kind == SV_G_U && is_phase_diag(g.m))) {
        it.diag = true;
        it.pivot = g.target;
        it.wbit = g.kind == SV_G_U ? -1 : g.control;
        const double theta = g.kind == SV_G_CPHASE ? g.m[0] : std::atan2(g.m[7], g.m[6]);
        it.turn = angle_to_turn(theta);
        it.qmask = tb | (it.wbit >= 0 ? uint64_t(1) << it.wbit : 0);
        return it;
    }
    it.target = g.target;
    it.control = g.kind == SV_G_U ? -1 : g.control;
    it.swap = is_pauli_x(g.m);
    std::memcpy(it.m, g.m, sizeof it.m);
    it.qmask = tb | (it.control >= 0 ? uint64_t(1) << it.control : 0);
    return it;
}

// Emits the pending diagonal terms that touch any qubit of `qm` (all of them
// when qm is ~0) as one diagonal op appended to `ops`.
void flush_diag(std::map<int, PPivot> &pending, uint64_t qm, std::vector<POp> &ops)
{
    std::vector<PPivot> out;
    for (auto it = pending.begin(); it != pending.end();) {
        PPivot &P = it->second;
        PPivot part;
        part.p = P.p;
        const bool whole = (qm >> P.p) & 1;
        std::vector<DTerm> keep;
        for (const DTerm &t : P.terms) {
            if (whole || (t.wbit >= 0 && ((qm >> t.wbit) & 1)))
                part.terms.push_back(t);
            else
                keep.push_back(t);
        }
        if (!part.terms.empty()) out.push_back(std::move(part));
        P.terms.swap(keep);
        if (P.terms.empty())
            it = pending.erase(it);
        else
            ++it;
    }
    if (!out.empty()) {
        POp op;
        op.kind = TOP_DIAG;
        for (PPivot &P : out) {
            for (const DTerm &t : P.terms) op.gates.push_back(t.gate);
            op.piv.push_back(std::move(P));
        }
        ops.push_back(std::move(op));
    }
}

// Register groups of one pass, by the light-cone rule: a group gets up to K
// register qubits (a target, both qubits of a 4x4, and a control when it is a
// tile qubit and fits), and takes every op whose register qubits it holds and
// that touches no qubit of an op left for a later group. Diagonal ops need no
// register qubit. Ops only move ahead of ops on other qubits. `ops` are in
// storage bits; T is the tile's storage bits (ascending) and Pm their mask.
// With `spread`, two-qubit blocks are formed over the whole pass first (so a
// block is not cut where one group's light cone ends) with the spread rule of
// fuse_group.
//
// With `cover`, each group instead takes the register set under which the most
// op cost can run next: sets of K qubits drawn from the qubits of the first
// ops left (targets, both qubits of 4x4s, tile controls) are scored by
// running the light-cone rule with the set fixed, the first-fit set among
// them, and the best is kept.
std::vector<PGroup> make_groups(std::vector<POp> ops, uint64_t Pm, const std::vector<int> &T,
                                const TileGeom &geo, bool spread, bool cover = false)
{
    auto local = [&](int b) { return int(std::lower_bound(T.begin(), T.end(), b) - T.begin()); };
    if (spread) ops = fuse_group(std::move(ops), Pm, true);
    std::vector<uint64_t> qmask(ops.size());
    std::vector<int> rest(ops.size()), later;
    for (size_t i = 0; i < ops.size(); ++i) {
        qmask[i] = op_qmask(ops[i]);
        rest[i] = int(i);
    }
    auto need_of = [&](int i) {
        const POp &op = ops[i];
        return op.kind == TOP_U4 ? qmask[i] : uint64_t(1) << op.target;
    };
    // Op cost that runs with register set S fixed (the light-cone rule).
    auto coverage = [&](uint64_t S) {
        uint64_t blocked = 0;
        double score = 0;
        for (int i : rest) {
            if ((blocked & Pm) == Pm) break;
            const uint64_t qm = qmask[i];
            if (qm & blocked) {
                blocked |= qm;
                continue;
            }
            const POp &op = ops[i];
            if (op.kind != TOP_DIAG && (need_of(i) & ~S)) {
                blocked |= qm;
                continue;
            }
            score += op_cost(op);
        }
        return score;
    };
    std::vector<PGroup> groups;
    while (!rest.empty()) {
        PGroup cur;
        uint64_t Sq = 0, blocked = 0;
        later.clear();
        uint64_t fixed = 0;   // cover: the chosen register set
        if (cover) {
            // First-fit set (as below) and the candidate pool.
            uint64_t ff = 0, pool = 0, blk = 0;
            for (int i : rest) {
                const uint64_t qm = qmask[i];
                if (qm & blk) {
                    blk |= qm;
                    continue;
                }
                if (ops[i].kind == TOP_DIAG) continue;
                const uint64_t need = need_of(i);
                if (__builtin_popcountll(ff | need) <= geo.K) ff |= need;
                else blk |= qm;
                uint64_t q = need;
                if (ops[i].kind != TOP_U4 && ops[i].control >= 0 && ((Pm >> ops[i].control) & 1))
                    q |= uint64_t(1) << ops[i].control;
                if (__builtin_popcountll(pool | q) > kCoverPool) break;
                pool |= q;
            }
            fixed = ff;
            double best = coverage(ff);
            int pb[64], np = 0;
            for (int b = 0; b < 64; ++b)
                if ((pool >> b) & 1) pb[np++] = b;
            const int want = std::min(geo.K, np);
            for (uint32_t m = 1; m < (1u << np); ++m) {
                if (__builtin_popcount(m) != want) continue;
                uint64_t S = 0;
                for (int k = 0; k < np; ++k)
                    if ((m >> k) & 1) S |= uint64_t(1) << pb[k];
                const double sc = coverage(S);
                if (sc > best) {
                    best = sc;
                    fixed = S;
                }
            }
            Sq = fixed;
        }
        for (size_t k = 0; k < rest.size(); ++k) {
            const int i = rest[k];
            POp &op = ops[i];
            const uint64_t qm = qmask[i];
            if ((blocked & Pm) == Pm) {   // nothing later can join
                later.insert(later.end(), rest.begin() + long(k), rest.end());
                break;
            }
            if (qm & blocked) {
                blocked |= qm;
                later.push_back(i);
                continue;
            }
            if (op.kind == TOP_DIAG) {
                cur.ops.push_back(std::move(op));
                continue;
            }
            const uint64_t need = op.kind == TOP_U4 ? qm : uint64_t(1) << op.target;
            uint64_t want = need;
            if (op.kind != TOP_U4 && op.control >= 0 && !op.xcm && ((Pm >> op.control) & 1))
                want |= uint64_t(1) << op.control;
            if (cover) {
                if (need & ~fixed) {
                    blocked |= qm;
                    later.push_back(i);
                    continue;
                }
            } else if (__builtin_popcountll(Sq | want) <= geo.K) {
                Sq |= want;
            } else if (__builtin_popcountll(Sq | need) <= geo.K) {
                Sq |= need;
            } else {
                blocked |= qm;
                later.push_back(i);
                continue;
            }
            cur.ops.push_back(std::move(op));
        }
        for (int b = 0; b < 64; ++b)
            if ((Sq >> b) & 1) cur.S.push_back(local(b));
        groups.push_back(std::move(cur));
        rest.swap(later);
    }
    for (PGroup &g : groups) {
        // Pad S with the highest unused local bits so the threads of a
        // wave differ in low local bits (contiguous LDS slots).
        for (int b = geo.L - 1; b >= 0 && int(g.S.size()) < geo.K; --b)
            if (std::find(g.S.begin(), g.S.end(), b) == g.S.end()) g.S.push_back(b);
        std::sort(g.S.begin(), g.S.end());
        if (geo.fuse4 && geo.K >= 2) {
            uint64_t regq = 0;
            for (int sidx : g.S) regq |= uint64_t(1) << T[sidx];
            g.ops = fuse_group(std::move(g.ops), regq, spread);
        }
        if (geo.K == kTileMaxK) fold_exit(g, T);
    }
    return groups;
}

double groups_cost(const std::vector<PGroup> &groups)
{
    double c = kGroupCost * double(groups.size());
    for (const PGroup &g : groups)
        for (const POp &op : g.ops) c += op_cost(op);
    return c;
}

// Splits the items into passes. *ok is false if some item could not be
// placed (the geometry left no free tile bit); the plan is then incomplete.
//
// With `relabel`, each pass also chooses the storage order it leaves behind:
// the index bits 0..nlow-1, which every tile must hold (whole 128-byte
// lines), receive tile qubits that the next gates need, instead of always
// holding qubits 0..nlow-1. The last pass (or, when it cannot, extra passes
// without gates) returns the state to the standard order.
std::vector<PPass> plan_passes_one(int n, const TileGeom &geo, const std::vector<Item> &items,
                                   bool *ok, bool relabel)
{
    *ok = true;
    std::vector<PPass> passes;
    // Items still to place, as indices into `items`, in gate order.
    std::vector<int> rem(items.size());
    for (size_t k = 0; k < items.size(); ++k) rem[k] = int(k);
    Layout lay(n);
    int restores = 0;
    while (!rem.empty() || !lay.identity()) {
        if (rem.empty() && ++restores > 2 * n + 2) {   // cannot happen: each restore fixes a qubit
            *ok = false;
            break;
        }
        uint64_t Tm = 0;   // logical qubits of the tile
        int tcount = 0;
        for (int b = 0; b < geo.nlow; ++b) {
            Tm |= uint64_t(1) << lay.inv[b];
            ++tcount;
        }
        uint64_t blocked = 0;
        std::vector<int> next;
        std::vector<POp> ops;
        std::map<int, PPivot> pending;
        const uint64_t all = n >= 64 ? ~uint64_t(0) : (uint64_t(1) << n) - 1;
        for (size_t ii = 0; ii < rem.size(); ++ii) {
            const Item &it = items[rem[ii]];
            if (blocked == all) {   // nothing later can join this pass
                next.insert(next.end(), rem.begin() + long(ii), rem.end());
                break;
            }
            if (it.qmask & blocked) {
                next.push_back(rem[ii]);
                blocked |= it.qmask;
                continue;
            }
            if (it.diag) {
                // A pair term needs one of its qubits in the tile (the device
                // form has no term on two bits of the tile index).
                if (it.wbit >= 0 && !((Tm >> it.pivot) & 1) && !((Tm >> it.wbit) & 1)) {
                    if (tcount < geo.L) {
                        Tm |= uint64_t(1) << it.pivot;
                        ++tcount;
                    } else {
                        next.push_back(rem[ii]);
                        blocked |= it.qmask;
                        continue;
                    }
                }
                PPivot &P = pending[it.pivot];
                P.p = it.pivot;
                P.terms.push_back(DTerm{it.wbit, it.turn, it.gate});
                continue;
            }
            if (!((Tm >> it.target) & 1)) {
                if (tcount < geo.L) {
                    Tm |= uint64_t(1) << it.target;
                    ++tcount;
                } else {
                    next.push_back(rem[ii]);
                    blocked |= it.qmask;
                    continue;
                }
            }
            flush_diag(pending, it.qmask, ops);
            POp op;
            op.kind = it.swap ? TOP_SWAP : TOP_U;
            op.target = it.target;
            op.control = it.control;
            op.xcm = it.xcm;
            std::memcpy(op.m, it.m, sizeof op.m);
            op.gates.push_back(it.gate);
            ops.push_back(std::move(op));
        }
        flush_diag(pending, ~uint64_t(0), ops);
        if (ops.empty() && !rem.empty()) {   // no progress: refuse rather than drop gates
            *ok = false;
            break;
        }
        auto take = [&](int q) {
            if (tcount < geo.L && !((Tm >> q) & 1)) {
                Tm |= uint64_t(1) << q;
                ++tcount;
            }
        };
        const bool last = next.empty();
        if (relabel) {
            if (last) {
                // Room left goes to the qubits out of their home bits.
                for (int q : cycle_order(lay, geo.nlow)) take(q);
            } else {
                // Room left goes to the qubits the next gates touch, so that
                // they can be left in the low index bits.
                for (int idx : next) {
                    const Item &it = items[idx];
                    if (tcount >= geo.L) break;
                    for (uint64_t m = it.qmask; m; m &= m - 1) take(__builtin_ctzll(m));
                }
            }
        }
        // Fill T up to L qubits with the lowest unused ones.
        for (int b = 0; b < n && tcount < geo.L; ++b) take(b);
        PPass pass;
        uint64_t Pm = 0;   // the tile's index bits in storage
        for (int q = 0; q < n; ++q)
            if ((Tm >> q) & 1) Pm |= uint64_t(1) << lay.pos[q];
        for (int b = 0; b < n; ++b)
            if ((Pm >> b) & 1) pass.T.push_back(b);
        for (POp &op : ops) to_storage(op, lay.pos);
        auto local = [&](int b) {
            return int(std::lower_bound(pass.T.begin(), pass.T.end(), b) - pass.T.begin());
        };
        if (relabel) {
            // The storage order this pass leaves: first the qubits wanted in
            // the low bits (the next gates' qubits among the tile's, in gate
            // order; none after the last pass), then every other tile qubit at
            // its home bit if the tile holds that bit, else where it was, else
            // anywhere free in the tile.
            std::vector<int> want;
            if (!last) {
                for (int idx : next) {
                    const Item &it = items[idx];
                    for (uint64_t m = it.qmask & Tm; m && int(want.size()) < geo.nlow; m &= m - 1) {
                        const int q = __builtin_ctzll(m);
                        if (std::find(want.begin(), want.end(), q) == want.end()) want.push_back(q);
                    }
                    if (int(want.size()) >= geo.nlow) break;
                }
                for (int b = 0; b < geo.nlow && int(want.size()) < geo.nlow; ++b)
                    if (std::find(want.begin(), want.end(), lay.inv[b]) == want.end())
                        want.push_back(lay.inv[b]);
            }
            std::vector<int> np(n, -1);
            std::vector<char> used(n, 0);
            auto place = [&](int q, int b) {
                np[q] = b;
                used[b] = 1;
            };
            for (int q : want)
                if (q < geo.nlow) place(q, q);
            for (int q : want)
                if (np[q] < 0 && lay.pos[q] < geo.nlow && !used[lay.pos[q]]) place(q, lay.pos[q]);
            for (int q : want)
                if (np[q] < 0)
                    for (int b = 0; b < geo.nlow; ++b)
                        if (!used[b]) {
                            place(q, b);
                            break;
                        }
            for (int q = 0; q < n; ++q)
                if (((Tm >> q) & 1) && np[q] < 0 && ((Pm >> q) & 1) && !used[q] &&
                    (q >= geo.nlow || want.empty()))
                    place(q, q);
            for (int q = 0; q < n; ++q)
                if (((Tm >> q) & 1) && np[q] < 0 && !used[lay.pos[q]] &&
                    (lay.pos[q] >= geo.nlow || want.empty()))
                    place(q, lay.pos[q]);
            for (int q = 0; q < n; ++q)
                if (((Tm >> q) & 1) && np[q] < 0)
                    for (int b : pass.T)
                        if (!used[b]) {
                            place(q, b);
                            break;
                        }
            pass.osrc.assign(geo.L, 0);
            bool moved = false;
            for (int q = 0; q < n; ++q)
                if ((Tm >> q) & 1) {
                    pass.osrc[local(np[q])] = local(lay.pos[q]);
                    moved |= np[q] != lay.pos[q];
                }
            for (int q = 0; q < n; ++q)
                if ((Tm >> q) & 1) {
                    lay.pos[q] = np[q];
                    lay.inv[np[q]] = q;
                }
            if (!moved) pass.osrc.clear();
        }
        // Groups, made each way; the cheapest set is kept. The coverage
        // search (fewer groups: 93 -> 72 on the 30-qubit layered circuit,
        // 2-4 % of its time) costs host time per group, so it runs only for
        // states whose passes are long enough to repay it.
        {
            const bool try_cover = n >= kCoverMinQubits;
            std::vector<PGroup> ga;
            double best = 0;
            for (int w = 0; w < 4; ++w) {
                const bool spread = w & 1, cover = w & 2;
                if (cover && !try_cover) continue;
                if (spread && !(geo.fuse4 && geo.K >= 2)) continue;
                std::vector<PGroup> gw = make_groups(ops, Pm, pass.T, geo, spread, cover);
                const double c = groups_cost(gw);
                if (ga.empty() || c < best) {
                    best = c;
                    ga.swap(gw);
                }
            }
            pass.groups = std::move(ga);
        }
        passes.push_back(std::move(pass));
        rem.swap(next);
    }
    return passes;
}

// With `relabel`, both plans are made and the one with the lower estimated
// cost is kept (each pass costs the larger of its HBM time and its ops; a
// short circuit can lose more to the passes that restore the standard order
// than it gains).
std::vector<PPass> plan_passes(int n, const TileGeom &geo, const std::vector<Item> &items, bool *ok,
                               bool relabel = false)
{
    std::vector<PPass> fixed = plan_passes_one(n, geo, items, ok, false);
    if (!relabel || !*ok) return fixed;
    bool ok_r = true;
    std::vector<PPass> moved = plan_passes_one(n, geo, items, &ok_r, true);
    auto cost = [](const std::vector<PPass> &ps) {
        double c = 0;
        for (const PPass &p : ps) c += std::max(kPassFloor, groups_cost(p.groups));
        return c;
    };
    if (ok_r && cost(moved) < cost(fixed)) return moved;
    return fixed;
}

// plan_passes, and for a state past the last-level cache whose fixed low bits
// are the default, a second plan with kLongRunLow of them: each tile then
// reads and writes longer contiguous runs, which the memory serves faster
// (30 qubits, 4 passes of 8-9 groups: complex64 QFT 17.2 ms with runs of
// 128 B, 15.9 ms with 512 B), but the planner has fewer free tile qubits.
// The second plan is kept when it needs fewer passes, or as many and at most
// one group more; geo.nlow is then updated.
std::vector<PPass> plan_passes_geo(int n, TileGeom &geo, const std::vector<Item> &items, bool *ok,
                                   bool relabel)
{
    std::vector<PPass> base = plan_passes(n, geo, items, ok, relabel);
    const uint64_t bytes = (uint64_t(1) << n) * (geo.c64 ? 8 : 16);
    if (!*ok || !geo.nlow_free || bytes <= kStreamBytes || geo.L >= n) return base;
    TileGeom alt = geo;
    alt.nlow = std::min(kLongRunLow, geo.L - 1);
    if (alt.nlow <= geo.nlow) return base;
    bool ok_a = true;
    std::vector<PPass> other = plan_passes(n, alt, items, &ok_a, relabel);
    if (!ok_a) return base;
    auto groups = [](const std::vector<PPass> &ps) {
        size_t c = 0;
        for (const PPass &p : ps) c += p.groups.size();
        return c;
    };
    if (other.size() < base.size() ||
        (other.size() == base.size() && groups(other) <= groups(base) + 1)) {
        geo = alt;
        return other;
    }
    return base;
}

// ---- flattening and execution ---------------------------------------------

// Tables of a diagonal op in one group (the quadratic form described with
// TileOp): rows of the tile-independent turns for every thread, byte tables
// over the tile index for weights against qubits outside the tile, and the
// constant phases of the register-only terms. Returns false for a pair term
// on two qubits outside the tile (the planner never makes one).
bool diag_tables(const POp &op, const std::vector<int> &T, const std::vector<int> &S,
                 const int32_t *ns, int L, int K, uint64_t omask, std::vector<uint64_t> &dtab,
                 TileOp &to)
{
    auto lidx = [&](int q) {
        const auto it = std::lower_bound(T.begin(), T.end(), q);
        return (it != T.end() && *it == q) ? int(it - T.begin()) : -1;
    };
    auto opos = [&](int q) { return __builtin_popcountll(omask & ((uint64_t(1) << q) - 1)); };
    std::vector<uint64_t> a(L, 0), Q(size_t(L) * L, 0);
    std::vector<std::vector<uint64_t>> ow(L + 1);   // [tile bit, or L: one-qubit][outside position]
    int maxo = -1;
    auto add_ow = [&](int l, int o, uint64_t t) {
        if (int(ow[l].size()) <= o) ow[l].resize(o + 1, 0);
        ow[l][o] += t;
        maxo = std::max(maxo, o);
    };
    for (const PPivot &P : op.piv)
        for (const DTerm &t : P.terms) {
            const int lp = lidx(P.p);
            if (t.wbit < 0) {
                if (lp >= 0) a[lp] += t.turn;
                else add_ow(L, opos(P.p), t.turn);
                continue;
            }
            const int lw = lidx(t.wbit);
            if (lp >= 0 && lw >= 0) Q[size_t(std::min(lp, lw)) * L + std::max(lp, lw)] += t.turn;
            else if (lp >= 0) add_ow(lp, opos(t.wbit), t.turn);
            else if (lw >= 0) add_ow(lw, opos(P.p), t.turn);
            else return false;
        }
    auto q = [&](int l0, int l1) { return Q[size_t(std::min(l0, l1)) * L + std::max(l0, l1)]; };
    const double two_pi = 6.283185307179586476925286766559;
    bool any = false;
    for (int r = 0; r < 16; ++r) {
        uint64_t t = 0;
        if (r < (1 << K))
            for (int k = 0; k < K; ++k) {
                if (!((r >> k) & 1)) continue;
                t += a[S[k]];
                for (int k2 = k + 1; k2 < K; ++k2)
                    if ((r >> k2) & 1) t += q(S[k], S[k2]);
            }
        any |= t != 0;
        const double ang = two_pi * std::ldexp(double(t), -64);
        to.m4[2 * r] = t ? std::cos(ang) : 1.0;
        to.m4[2 * r + 1] = t ? std::sin(ang) : 0.0;
        to.mf4[2 * r] = float(to.m4[2 * r]);
        to.mf4[2 * r + 1] = float(to.m4[2 * r + 1]);
    }
    to.pj = any ? 1 : 0;
    const int nt = L - K;
    // The shape of the op: which coef_k, and whether base, can be non-zero
    // (their terms, as set up above: the thread rows below and the byte
    // tables of the outside weights).
    auto nonzero = [](const std::vector<uint64_t> &v) {
        return std::any_of(v.begin(), v.end(), [](uint64_t t) { return t != 0; });
    };
    to.dlin = nonzero(ow[L]) ? kDiagBase : 0u;
    for (int k = 0; k < nt; ++k) {
        if (a[ns[k]] || nonzero(ow[ns[k]])) to.dlin |= kDiagBase;
        for (int k2 = k + 1; k2 < nt; ++k2)
            if (q(ns[k], ns[k2])) to.dlin |= kDiagBase;
        for (int j = 0; j < K; ++j)
            if (q(ns[k], S[j])) to.dlin |= 1u << j;
    }
    for (int j = 0; j < K; ++j)
        if (nonzero(ow[S[j]])) to.dlin |= 1u << j;
    to.dthr = int(dtab.size());
    for (uint32_t tid = 0; tid < (1u << nt); ++tid) {
        uint64_t b0 = 0, cr[kTileMaxK] = {};
        for (int k = 0; k < nt; ++k) {
            if (!((tid >> k) & 1)) continue;
            b0 += a[ns[k]];
            for (int k2 = k + 1; k2 < nt; ++k2)
                if ((tid >> k2) & 1) b0 += q(ns[k], ns[k2]);
            for (int j = 0; j < K; ++j) cr[j] += q(ns[k], S[j]);
        }
        dtab.push_back(b0);
        for (int j = 0; j < K; ++j) dtab.push_back(cr[j]);
    }
    if (maxo < 0) {
        to.dout = -1;
        to.dbytes = 0;
        return true;
    }
    const int nb = maxo / 8 + 1;
    to.dout = int(dtab.size());
    to.dbytes = nb;
    for (int b = 0; b < nb; ++b)
        for (int l = 0; l <= L; ++l)
            for (int v = 0; v < 256; ++v) {
                uint64_t t = 0;
                for (int j = 0; j < 8; ++j) {
                    const int o = 8 * b + j;
                    if (((v >> j) & 1) && o < int(ow[l].size())) t += ow[l][o];
                }
                dtab.push_back(t);
            }
    return true;
}

// Thread bits of a register group: thread bit k is local tile bit ns[k],
// over the tile bits not in S. Complex128: 16-byte LDS accesses are free of
// bank conflicts when the slots of 16 neighbouring lanes differ modulo 16
// (reads) and of 8 modulo 8 (writes); in the slot map l + l/16 + l/256,
// local bit b adds 2^(b mod 4) modulo 16, so thread bits 0..3 take a free bit
// of class b mod 4 = 0, 1, 2, 3 (the lowest: the tile's low bits stay on the
// low thread bits, which keeps direct transfers coalesced), and the rest
// follow in ascending order. Complex64: ascending.
void thread_order(const std::vector<int> &S, const TileGeom &geo, int32_t *ns)
{
    std::vector<int> fr, order;
    for (int b = 0; b < geo.L; ++b)
        if (std::find(S.begin(), S.end(), b) == S.end()) fr.push_back(b);
    if (!geo.c64)
        for (int k = 0; k < 4 && int(order.size()) < int(fr.size()); ++k)
            for (int b : fr)
                if (b % 4 == k) {
                    order.push_back(b);
                    break;
                }
    for (int b : fr)
        if (std::find(order.begin(), order.end(), b) == order.end()) order.push_back(b);
    for (size_t k = 0; k < order.size(); ++k) ns[k] = order[k];
}

struct Flat {
    bool ok = true;                 // false: a diagonal pair term on two outside bits
    std::vector<TileGroup> groups;
    std::vector<TileOp> ops;
    std::vector<uint64_t> dtab;     // diagonal-op tables
    std::vector<TileArgs> args;   // one per pass (pointers patched after upload)
    std::vector<double> flops;    // per pass
};

Flat flatten(int n, const TileGeom &geo, const std::vector<PPass> &passes)
{
    Flat f;
    for (const PPass &pass : passes) {
        TileArgs a{};
        a.L = geo.L;
        a.nlow = geo.nlow;
        uint64_t Tm = 0;
        for (int b : pass.T) Tm |= uint64_t(1) << b;
        const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
        a.tmask = Tm;
        a.omask = all & ~Tm;
        a.nnon = n - geo.L;
        a.ntiles = uint64_t(1) << a.nnon;
        a.group0 = int(f.groups.size());
        a.ngroups = int(pass.groups.size());
        a.has_diag = 0;
        a.permute = pass.osrc.empty() ? 0 : 1;
        a.osrc = 0;
        for (int j = 0; j < int(pass.osrc.size()); ++j) a.osrc |= uint64_t(pass.osrc[j]) << (4 * j);
        double flops = 0;
        auto local = [&](int q) {
            return int(std::lower_bound(pass.T.begin(), pass.T.end(), q) - pass.T.begin());
        };
        const double N = std::ldexp(1.0, n);
        for (const PGroup &g : pass.groups) {
            TileGroup tg{};
            for (int k = 0; k < geo.K; ++k) tg.s[k] = g.S[k];
            thread_order(g.S, geo, tg.ns);
            tg.op0 = int(f.ops.size());
            tg.nops = int(g.ops.size());
            tg.has_exit = g.folded.empty() ? 0 : 1;
            tg.xb = g.xb;
            for (int k = 0; k < kTileMaxK; ++k) tg.xs[k] = g.xs[k];
            for (const POp &op : g.ops) {
                TileOp to{};
                to.kind = op.kind;
                to.lctrl = -1;
                to.octrl = -1;
                if (op.kind == TOP_DIAG) {
                    a.has_diag = 1;
                    if (!diag_tables(op, pass.T, g.S, tg.ns, geo.L, geo.K, a.omask, f.dtab, to))
                        f.ok = false;
                    flops += 12.0 * N;
                } else if (op.kind == TOP_U4) {
                    to.pj = int(std::find(g.S.begin(), g.S.end(), local(op.q0)) - g.S.begin());
                    to.pk = int(std::find(g.S.begin(), g.S.end(), local(op.q1)) - g.S.begin());
                    std::memcpy(to.m4, op.m4, sizeof to.m4);
                    for (int k = 0; k < 32; ++k) to.mf4[k] = float(op.m4[k]);
                    flops += 30.0 * N;   // 4 complex products and 3 sums per amplitude
                } else {
                    const int p = local(op.target);
                    to.pj = int(std::find(g.S.begin(), g.S.end(), p) - g.S.begin());
                    to.pk = -1;
                    if (op.xcm) {
                        // several controls: masks of the tile-bit and the
                        // outside controls, tested per amplitude and per tile
                        const uint64_t cm = op.xcm | (uint64_t(1) << op.control);
                        for (uint64_t m = cm & Tm; m; m &= m - 1)
                            to.lcm |= 1u << local(__builtin_ctzll(m));
                        to.ocm = cm & ~Tm;
                    } else if (op.control >= 0) {
                        if ((Tm >> op.control) & 1) {
                            to.lctrl = local(op.control);
                            const int pc = int(std::find(g.S.begin(), g.S.end(), to.lctrl) - g.S.begin());
                            if (pc < geo.K) to.pk = pc;
                        } else {
                            to.octrl = op.control;
                        }
                    }
                    std::memcpy(to.m, op.m, sizeof to.m);
                    for (int k = 0; k < 8; ++k) to.mf[k] = float(op.m[k]);
                    const int nctrl = (op.control >= 0 ? 1 : 0) + __builtin_popcountll(op.xcm);
                    if (op.kind == TOP_U) flops += std::ldexp(14.0 * N, -nctrl);
                }
                f.ops.push_back(to);
            }
            f.groups.push_back(tg);
        }
        f.args.push_back(a);
        f.flops.push_back(flops);
    }
    return f;
}

template <typename A>
void fill_phase_table(A *tab)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < 256; ++k) {
        const double a1 = two_pi * (double(k) / 256.0);
        const double a2 = two_pi * (double(k) / 65536.0);
        tab[k].x = std::cos(a1);
        tab[k].y = std::sin(a1);
        tab[256 + k].x = std::cos(a2);
        tab[256 + k].y = std::sin(a2);
    }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- dense 5-qubit blocks (SV_FUSE_DENSE) ------------------------------------

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Control qubits of a validated gate record, as a mask.
uint64_t gate_cmask(const sv_gate &g)
{
    if (g.kind == SV_G_MCU) return uint64_t(uint32_t(g.control)) | (uint64_t(uint32_t(g.flags)) << 32);
    return g.kind == SV_G_U ? 0 : uint64_t(1) << g.control;
}

uint64_t gate_qmask(const sv_gate &g) { return (uint64_t(1) << g.target) | gate_cmask(g); }

struct DBlock {
    uint64_t qmask = 0;
    std::vector<int> gates;
};

// Groups the gates into blocks of at most five qubits. A gate joins the open
// block when the union stays within five qubits and it touches no qubit of a
// gate already left for a later block (those commute past it).
std::vector<DBlock> plan_dense(int n, const sv_gate *g, size_t ng)
{
    std::vector<DBlock> blocks;
    std::vector<int> rem(ng);
    for (size_t i = 0; i < ng; ++i) rem[i] = int(i);
    while (!rem.empty()) {
        DBlock b;
        uint64_t blocked = 0;
        std::vector<int> next;
        for (int i : rem) {
            const uint64_t qm = gate_qmask(g[i]);
            if ((qm & blocked) || popcount64(b.qmask | qm) > 5) {
                next.push_back(i);
                blocked |= qm;
                continue;
            }
            b.qmask |= qm;
            b.gates.push_back(i);
        }
        // Pad to five qubits with the highest unused ones, so that the low
        // index bits stay in the column index (coalesced columns).
        for (int q = n - 1; q >= 0 && popcount64(b.qmask) < 5; --q) b.qmask |= uint64_t(1) << q;
        blocks.push_back(std::move(b));
        rem.swap(next);
    }
    return blocks;
}

// The block's 32x32 complex matrix (FP64), built by applying each gate's
// stride update to the 32 columns of the identity, then written as the real
// 64x64 form [[Re, -Im], [Im, Re]] in row-major order.
template <typename R>
void block_matrix(const DBlock &b, const sv_gate *g, R *out)
{
    int pos[64];
    int k = 0;
    for (int q = 0; q < 64; ++q)
        if ((b.qmask >> q) & 1) pos[q] = k++;
    static thread_local double re[32][32], im[32][32];   // [row][column]
    for (int i = 0; i < 32; ++i)
        for (int j = 0; j < 32; ++j) {
            re[i][j] = i == j ? 1.0 : 0.0;
            im[i][j] = 0.0;
        }
    for (int gi : b.gates) {
        const sv_gate &G = g[gi];
        double m[8];
        if (G.kind == SV_G_CPHASE) {
            const double c = std::cos(G.m[0]), s_ = std::sin(G.m[0]);
            const double d[8] = {1, 0, 0, 0, 0, 0, c, s_};
            std::memcpy(m, d, sizeof m);
        } else {
            std::memcpy(m, G.m, sizeof m);
        }
        const int t = pos[G.target];
        int cm = 0;   // the controls as local bits: the update runs where all are 1
        for (uint64_t x = gate_cmask(G); x; x &= x - 1) cm |= 1 << pos[__builtin_ctzll(x)];
        for (int col = 0; col < 32; ++col)
            for (int i0 = 0; i0 < 32; ++i0) {
                if ((i0 >> t) & 1) continue;
                if ((i0 & cm) != cm) continue;
                const int i1 = i0 | (1 << t);
                const double ar = re[i0][col], ai = im[i0][col];
                const double br = re[i1][col], bi = im[i1][col];
                re[i0][col] = m[0] * ar - m[1] * ai + m[2] * br - m[3] * bi;
                im[i0][col] = m[0] * ai + m[1] * ar + m[2] * bi + m[3] * br;
                re[i1][col] = m[4] * ar - m[5] * ai + m[6] * br - m[7] * bi;
                im[i1][col] = m[4] * ai + m[5] * ar + m[6] * bi + m[7] * br;
            }
    }
    for (int i = 0; i < 32; ++i)
        for (int j = 0; j < 32; ++j) {
            out[i * 64 + j] = R(re[i][j]);
            out[i * 64 + 32 + j] = R(-im[i][j]);
            out[(32 + i) * 64 + j] = R(im[i][j]);
            out[(32 + i) * 64 + 32 + j] = R(re[i][j]);
        }
}

}  // namespace

// Device resources of the planner, owned by a state handle.
struct PlanCache {
    void *dev = nullptr;
    size_t dev_cap = 0;
    void *host = nullptr;       // pinned staging
    size_t host_cap = 0;
    hipEvent_t staged = nullptr;
};

static PlanCache *cache_of(sv_state s)
{
    if (!s->plan) s->plan = new PlanCache();
    return static_cast<PlanCache *>(s->plan);
}

// Copies `bytes` of host data to the handle's device plan buffer through a
// pinned staging buffer, in stream order. Returns the device address.
static sv_status stage_upload(sv_state s, size_t bytes, const std::function<void(char *)> &fill,
                              char **dev_out, std::string *err)
{
    PlanCache *pc = cache_of(s);
    hipError_t e = hipSuccess;
    if (pc->staged) {
        e = hipEventSynchronize(pc->staged);   // staging buffer free again
        if (e != hipSuccess) { *err = hipGetErrorString(e); return SV_EDEVICE; }
    } else if ((e = hipEventCreateWithFlags(&pc->staged, hipEventDisableTiming)) != hipSuccess) {
        *err = hipGetErrorString(e);
        return SV_EDEVICE;
    }
    const size_t total = align_up(bytes, 256);
    if (pc->host_cap < total) {
        if (pc->host) (void)hipHostFree(pc->host);
        pc->host = nullptr;
        pc->host_cap = 0;
        if ((e = hipHostMalloc(&pc->host, total, 0)) != hipSuccess) {
            *err = "pinned staging allocation failed";
            return SV_ENOMEM;
        }
        pc->host_cap = total;
    }
    if (pc->dev_cap < total) {
        if (pc->dev) (void)hipFree(pc->dev);   // hipFree waits for work that may use it
        pc->dev = nullptr;
        pc->dev_cap = 0;
        if ((e = hipMalloc(&pc->dev, total)) != hipSuccess) {
            (void)hipGetLastError();
            *err = "device plan allocation failed";
            return SV_ENOMEM;
        }
        pc->dev_cap = total;
    }
    fill(static_cast<char *>(pc->host));
    e = hipMemcpyAsync(pc->dev, pc->host, total, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipEventRecord(pc->staged, s->stream);
    if (e != hipSuccess) { *err = hipGetErrorString(e); return SV_EDEVICE; }
    *dev_out = static_cast<char *>(pc->dev);
    return SV_OK;
}

// A gate list planned into tile passes, with the layout of what the passes
// read from device memory: groups | ops | diagonal tables | phase table.
struct TileRun {
    TileGeom geo;
    Flat f;
    size_t off_ops = 0, off_dtab = 0, off_tab = 0, total = 0;
};

static sv_status tile_plan(sv_state s, const sv_gate *gates, size_t n_gates, bool relabel,
                           TileRun *r, std::string *err)
{
    r->geo = geometry(s->n, s->dt, 0, s);
    std::vector<Item> items;
    items.reserve(n_gates);
    for (size_t i = 0; i < n_gates; ++i) items.push_back(classify(gates[i], int(i)));
    bool ok = true;
    const std::vector<PPass> passes = plan_passes_geo(s->n, r->geo, items, &ok, relabel);
    if (!ok) {
        *err = "planner could not place every gate with this tile geometry";
        return SV_EUNSUPPORTED;
    }
    r->f = flatten(s->n, r->geo, passes);
    if (!r->f.ok) {
        *err = "planner left a diagonal pair term outside the tile";
        return SV_EUNSUPPORTED;
    }
    const bool c64 = s->dt == SV_C64;
    const size_t tab_bytes = 512 * (c64 ? sizeof(float2) : sizeof(double2));
    r->off_ops = align_up(r->f.groups.size() * sizeof(TileGroup), 256);
    r->off_dtab = align_up(r->off_ops + r->f.ops.size() * sizeof(TileOp), 256);
    r->off_tab = align_up(r->off_dtab + r->f.dtab.size() * sizeof(uint64_t), 256);
    r->total = r->off_tab + tab_bytes;
    return SV_OK;
}

static void tile_fill(const TileRun &r, bool c64, char *h)
{
    std::memcpy(h, r.f.groups.data(), r.f.groups.size() * sizeof(TileGroup));
    std::memcpy(h + r.off_ops, r.f.ops.data(), r.f.ops.size() * sizeof(TileOp));
    std::memcpy(h + r.off_dtab, r.f.dtab.data(), r.f.dtab.size() * sizeof(uint64_t));
    if (c64) fill_phase_table(reinterpret_cast<float2 *>(h + r.off_tab));
    else fill_phase_table(reinterpret_cast<double2 *>(h + r.off_tab));
}

// Pass p's kernel arguments, with its tables at device address d.
static TileArgs tile_args(const TileRun &r, size_t p, void *psi, char *d)
{
    TileArgs a = r.f.args[p];
    a.psi = psi;
    a.groups = reinterpret_cast<const TileGroup *>(d);
    a.ops = reinterpret_cast<const TileOp *>(d + r.off_ops);
    a.dtab = reinterpret_cast<const uint64_t *>(d + r.off_dtab);
    a.phase_tab = d + r.off_tab;
    return a;
}

static sv_status run_tiles(sv_state s, const sv_gate *gates, size_t n_gates, bool relabel,
                           bool jit, std::string *err)
{
    TileRun r;
    if (sv_status st = tile_plan(s, gates, n_gates, relabel, &r, err)) return st;
    const bool c64 = s->dt == SV_C64;
    std::vector<JitKernel> kern;
    if (jit)
        if (sv_status st = jit_passes(s->dt, r.geo.K, r.f.args, r.f.groups, r.f.ops, &kern, err))
            return st;
    char *d = nullptr;
    sv_status st = stage_upload(s, r.total, [&](char *h) { tile_fill(r, c64, h); }, &d, err);
    if (st != SV_OK) return st;

    const double bytes = 2.0 * std::ldexp(1.0, s->n) * elem_bytes(s->dt);
    for (size_t p = 0; p < r.f.args.size(); ++p) {
        const TileArgs a = tile_args(r, p, s->psi, d);
        const int tok = prof_begin(s);
        hipError_t e = jit ? jit_launch(kern[p], a, r.geo.K, c64, s->stream)
                           : launch_tile(a, r.geo.K, c64, s->stream);
        prof_end(s, tok, KC_TILE, bytes, r.f.flops[p]);
        if (e != hipSuccess) { *err = std::string("tile launch: ") + hipGetErrorString(e); return SV_EDEVICE; }
    }
    return SV_OK;
}

sv_status tiles_prepare(sv_state s, const sv_gate *gates, size_t n_gates, bool relabel, void **dev,
                        std::vector<TileArgs> *launches, int *K, std::vector<JitKernel> *jit,
                        std::string *err)
{
    TileRun r;
    if (sv_status st = tile_plan(s, gates, n_gates, relabel, &r, err)) return st;
    if (jit)
        if (sv_status st = jit_passes(s->dt, r.geo.K, r.f.args, r.f.groups, r.f.ops, jit, err))
            return st;
    std::vector<char> h(r.total);
    tile_fill(r, s->dt == SV_C64, h.data());
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, r.total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dev = nullptr;
        *err = "device allocation of the tile plan failed";
        return SV_ENOMEM;
    }
    e = hipMemcpy(*dev, h.data(), r.total, hipMemcpyHostToDevice);   // synchronous, once
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        *err = hipGetErrorString(e);
        return SV_EDEVICE;
    }
    launches->clear();
    for (size_t p = 0; p < r.f.args.size(); ++p)
        launches->push_back(tile_args(r, p, s->psi, static_cast<char *>(*dev)));
    *K = r.geo.K;
    return SV_OK;
}

static sv_status run_dense(sv_state s, const sv_gate *gates, size_t n_gates, std::string *err)
{
    const std::vector<DBlock> blocks = plan_dense(s->n, gates, n_gates);
    const bool c64 = s->dt == SV_C64;
    const size_t mat_bytes = 64 * 64 * (c64 ? sizeof(float) : sizeof(double));
    char *d = nullptr;
    sv_status st = stage_upload(s, blocks.size() * mat_bytes, [&](char *h) {
        for (size_t b = 0; b < blocks.size(); ++b) {
            if (c64) block_matrix(blocks[b], gates, reinterpret_cast<float *>(h + b * mat_bytes));
            else block_matrix(blocks[b], gates, reinterpret_cast<double *>(h + b * mat_bytes));
        }
    }, &d, err);
    if (st != SV_OK) return st;
    const uint64_t all = (uint64_t(1) << s->n) - 1;
    const double N = std::ldexp(1.0, s->n);
    for (size_t b = 0; b < blocks.size(); ++b) {
        DenseArgs a{};
        a.psi = s->psi;
        a.mat = d + b * mat_bytes;
        a.bmask = blocks[b].qmask;
        a.omask = all & ~blocks[b].qmask;
        a.ncols = uint64_t(1) << (s->n - 5);
        const int tok = prof_begin(s);
        hipError_t e = launch_dense5(a, c64, s->stream);
        prof_end(s, tok, KC_DENSE, 2.0 * N * elem_bytes(s->dt), 256.0 * N);
        if (e != hipSuccess) { *err = std::string("dense launch: ") + hipGetErrorString(e); return SV_EDEVICE; }
    }
    return SV_OK;
}

sv_status dense_prepare(sv_state s, const sv_gate *gates, size_t n_gates, void **dev,
                        std::vector<DenseArgs> *launches, std::string *err)
{
    const std::vector<DBlock> blocks = plan_dense(s->n, gates, n_gates);
    const bool c64 = s->dt == SV_C64;
    const size_t mat_bytes = 64 * 64 * (c64 ? sizeof(float) : sizeof(double));
    std::vector<char> h(std::max<size_t>(blocks.size(), 1) * mat_bytes);
    for (size_t b = 0; b < blocks.size(); ++b) {
        if (c64) block_matrix(blocks[b], gates, reinterpret_cast<float *>(h.data() + b * mat_bytes));
        else block_matrix(blocks[b], gates, reinterpret_cast<double *>(h.data() + b * mat_bytes));
    }
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, h.size());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dev = nullptr;
        *err = "device allocation of the dense blocks failed";
        return SV_ENOMEM;
    }
    e = hipMemcpy(*dev, h.data(), h.size(), hipMemcpyHostToDevice);   // synchronous, once
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        *err = hipGetErrorString(e);
        return SV_EDEVICE;
    }
    const uint64_t all = (uint64_t(1) << s->n) - 1;
    launches->clear();
    for (size_t b = 0; b < blocks.size(); ++b) {
        DenseArgs a{};
        a.psi = s->psi;
        a.mat = static_cast<char *>(*dev) + b * mat_bytes;
        a.bmask = blocks[b].qmask;
        a.omask = all & ~blocks[b].qmask;
        a.ncols = uint64_t(1) << (s->n - 5);
        launches->push_back(a);
    }
    return SV_OK;
}

sv_status apply_unitary(sv_state s, const int32_t *q, int k, const double *u, std::string *err)
{
    const bool c64 = s->dt == SV_C64;
    const int dim = 1 << k;
    const uint64_t all = (uint64_t(1) << s->n) - 1;
    uint64_t qm = 0;
    for (int m = 0; m < k; ++m) qm |= uint64_t(1) << q[m];
    if (s->n < 9) {
        char *d = nullptr;
        const size_t bytes = size_t(dim) * dim * 2 * sizeof(double);
        sv_status st = stage_upload(s, bytes, [&](char *h) { std::memcpy(h, u, bytes); }, &d, err);
        if (st != SV_OK) return st;
        SmallUArgs a{};
        a.psi = s->psi;
        a.mat = d;
        a.omask = all & ~qm;
        a.ngroups = uint64_t(1) << (s->n - k);
        a.dim = dim;
        for (int c = 0; c < dim; ++c) {
            a.off[c] = 0;
            for (int m = 0; m < k; ++m)
                if ((c >> m) & 1) a.off[c] |= uint64_t(1) << q[m];
        }
        const int tok = prof_begin(s);
        hipError_t e = launch_unitary_small(a, c64, s->stream);
        prof_end(s, tok, KC_DENSE, 2.0 * std::ldexp(1.0, s->n) * elem_bytes(s->dt),
                 8.0 * dim * std::ldexp(1.0, s->n));
        if (e != hipSuccess) { *err = std::string("unitary launch: ") + hipGetErrorString(e); return SV_EDEVICE; }
        return SV_OK;
    }
    // Pad to five qubits with the highest unused ones (the low index bits stay
    // in the column index), then write U in the block's ascending bit order:
    // block row R holds U[r][c] when the padding bits of R and C agree.
    uint64_t bm = qm;
    for (int b = s->n - 1; b >= 0 && popcount64(bm) < 5; --b) bm |= uint64_t(1) << b;
    int pos[64];
    for (int b = 0, j = 0; b < 64; ++b)
        if ((bm >> b) & 1) pos[b] = j++;
    int lbit[5];                 // block bit of local bit m of U
    uint32_t padm = 0;           // block bits that are padding
    for (int m = 0; m < k; ++m) lbit[m] = pos[q[m]];
    for (int b = 0; b < 64; ++b)
        if (((bm >> b) & 1) && !((qm >> b) & 1)) padm |= 1u << pos[b];
    auto local = [&](int R) {
        int r = 0;
        for (int m = 0; m < k; ++m) r |= ((R >> lbit[m]) & 1) << m;
        return r;
    };
    const size_t mat_bytes = 64 * 64 * (c64 ? sizeof(float) : sizeof(double));
    auto fill = [&](char *h) {
        for (int R = 0; R < 32; ++R)
            for (int C = 0; C < 32; ++C) {
                double re = 0.0, im = 0.0;
                if ((R & padm) == (C & padm)) {
                    const int r = local(R), c = local(C);
                    re = u[2 * (r * dim + c)];
                    im = u[2 * (r * dim + c) + 1];
                }
                const double v[4] = {re, -im, im, re};   // [[Re, -Im], [Im, Re]]
                const int idx[4] = {R * 64 + C, R * 64 + 32 + C, (32 + R) * 64 + C,
                                    (32 + R) * 64 + 32 + C};
                for (int z = 0; z < 4; ++z) {
                    if (c64) reinterpret_cast<float *>(h)[idx[z]] = float(v[z]);
                    else reinterpret_cast<double *>(h)[idx[z]] = v[z];
                }
            }
    };
    char *d = nullptr;
    sv_status st = stage_upload(s, mat_bytes, fill, &d, err);
    if (st != SV_OK) return st;
    DenseArgs a{};
    a.psi = s->psi;
    a.mat = d;
    a.bmask = bm;
    a.omask = all & ~bm;
    a.ncols = uint64_t(1) << (s->n - 5);
    const double N = std::ldexp(1.0, s->n);
    const int tok = prof_begin(s);
    hipError_t e = launch_dense5(a, c64, s->stream);
    prof_end(s, tok, KC_DENSE, 2.0 * N * elem_bytes(s->dt), 256.0 * N);
    if (e != hipSuccess) { *err = std::string("dense launch: ") + hipGetErrorString(e); return SV_EDEVICE; }
    return SV_OK;
}

sv_status plan_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                   std::string *err)
{
    // Dense blocks need at least 16 columns of 32 amplitudes (n >= 9); smaller
    // registers are fused into tiles instead.
    if ((flags & SV_FUSE_DENSE) && s->n >= 9) return run_dense(s, gates, n_gates, err);
    return run_tiles(s, gates, n_gates, !(flags & SV_NO_RELABEL), (flags & SV_JIT) != 0, err);
}

void plan_release(sv_state s)
{
    if (!s->plan) return;
    PlanCache *pc = static_cast<PlanCache *>(s->plan);
    if (pc->staged) (void)hipEventSynchronize(pc->staged);
    if (pc->dev) (void)hipFree(pc->dev);
    if (pc->host) (void)hipHostFree(pc->host);
    if (pc->staged) (void)hipEventDestroy(pc->staged);
    delete pc;
    s->plan = nullptr;
}

// Host-only view of a dense-block plan: block qubit masks and each block's
// 32x32 complex matrix (row major, interleaved re/im) for the first `cap`
// blocks; returns the number of blocks.
int plan_dense_inspect(int n, const sv_gate *gates, size_t n_gates, uint64_t *masks,
                       double *mats, int cap)
{
    const std::vector<DBlock> blocks = plan_dense(n, gates, n_gates);
    std::vector<double> real(64 * 64);
    for (int b = 0; b < int(blocks.size()) && b < cap; ++b) {
        if (masks) masks[b] = blocks[b].qmask;
        if (!mats) continue;
        block_matrix(blocks[b], gates, real.data());
        for (int i = 0; i < 32; ++i)
            for (int j = 0; j < 32; ++j) {
                mats[(size_t(b) * 1024 + i * 32 + j) * 2] = real[i * 64 + j];
                mats[(size_t(b) * 1024 + i * 32 + j) * 2 + 1] = real[(32 + i) * 64 + j];
            }
    }
    return int(blocks.size());
}

// Host-only view of a plan, for inspection and tests.
int plan_inspect(int n, sv_dtype dt, const sv_gate *gates, size_t n_gates, bool relabel,
                 int32_t *gate_op, int32_t *n_passes, int32_t *n_groups, int32_t *n_ops)
{
    TileGeom geo = geometry(n, dt);
    std::vector<Item> items;
    for (size_t i = 0; i < n_gates; ++i) items.push_back(classify(gates[i], int(i)));
    bool ok = true;
    const std::vector<PPass> passes = plan_passes_geo(n, geo, items, &ok, relabel);
    if (!ok) return -1;
    int32_t seq = 0, groups = 0;
    if (gate_op)
        for (size_t i = 0; i < n_gates; ++i) gate_op[i] = -1;
    for (const PPass &p : passes) {
        for (const PGroup &g : p.groups) {
            ++groups;
            for (const std::vector<POp> *list : {&g.ops, &g.folded})
                for (const POp &op : *list) {
                    if (gate_op)
                        for (int gi : op.gates) gate_op[gi] = std::max(gate_op[gi], seq);
                    ++seq;
                }
        }
    }
    if (n_passes) *n_passes = int32_t(passes.size());
    if (n_groups) *n_groups = groups;
    if (n_ops) *n_ops = seq;
    return 0;
}

int plan_jit_check(int n, sv_dtype dt, const sv_gate *gates, size_t n_gates, bool relabel,
                   int32_t *n_programs, std::string *err)
{
    TileGeom geo = geometry(n, dt);
    std::vector<Item> items;
    for (size_t i = 0; i < n_gates; ++i) items.push_back(classify(gates[i], int(i)));
    bool ok = true;
    const std::vector<PPass> passes = plan_passes_geo(n, geo, items, &ok, relabel);
    if (!ok) {
        *err = "planner could not place every gate with this tile geometry";
        return -1;
    }
    const Flat f = flatten(n, geo, passes);
    if (!f.ok) {
        *err = "planner left a diagonal pair term outside the tile";
        return -1;
    }
    return jit_compile_only(dt, geo.K, f.args, f.groups, f.ops, n_programs, err) ? 0 : -2;
}

}  // namespace svk

// ---- planned circuits and batched launches -----------------------------------

namespace svk {

int wall_clock_khz()
{
    static int khz = 0;
    if (khz == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
    }
    return khz;
}

}  // namespace svk

struct sv_plan_s {
    // Distinct for every plan the process creates (never reused, unlike the
    // address of a destroyed plan): what a batch's captured graph is keyed on.
    uint64_t serial = 0;
    sv_state st = nullptr;
    int n = 0;
    sv_dtype dt = SV_C128;
    std::vector<svk::TileArgs> passes;   // device pointers patched
    std::vector<double> flops;
    void *dev = nullptr;
};

// Device buffers of one prepared batch: tasks | passes | start clocks | end clocks.
struct BatchImage {
    void *dev = nullptr;
    size_t cap = 0;
    size_t off_pass = 0, off_start = 0, off_end = 0;
    std::vector<uint32_t> level0;      // first task of each level, plus the end
    std::vector<int32_t> task_circ;    // circuit of each task
    size_t count = 0;                  // circuits
    // Circuits run whole by the persistent launch (before the levels):
    // circuit index of each entry, and where its table and clocks sit in `dev`.
    std::vector<int32_t> pcirc;
    size_t off_circ = 0, off_pstart = 0, off_pend = 0;
    // Circuits run pass by pass with the single-state kernel (beside the
    // levels): circuit index, its passes in `spasses` from sfirst[k] (scount[k]
    // of them), and where its two clock stamps sit in `dev`.
    std::vector<int32_t> scirc, sfirst, scount;
    std::vector<svk::TileArgs> spasses;
    size_t off_sstart = 0, off_send = 0;
};

struct sv_batch_s {
    sv_dtype dt = SV_C64;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;     // private stream for graph capture
    hipStream_t side = nullptr;        // the persistent launch runs here, beside the levels
    hipEvent_t fork = nullptr, join = nullptr;
    int blocks_per_cu = 2;
    uint32_t tiles_per_task = 8;
    int32_t persist_tiles = 0;         // circuits of at most this many tiles per pass
                                       // run whole in the persistent launch (0: none)
    int32_t solo_tiles = 0;            // circuits of at least this many tiles per pass
                                       // run pass by pass on `solo` (0: none)
    hipStream_t solo = nullptr;
    hipEvent_t sfork = nullptr, sjoin = nullptr;
    BatchImage work;                   // runs without SV_GRAPH
    BatchImage gimg;                   // the captured graph's own buffers
    hipGraphExec_t gexec = nullptr;
    std::vector<uintptr_t> gkey;       // content the graph was captured for
    void *host = nullptr;              // pinned staging
    size_t host_cap = 0;
    hipEvent_t staged = nullptr;
    const BatchImage *last = nullptr;  // image of the last run (for sv_batch_times)
};

namespace {

sv_status berr(sv_status st, const std::string &m) { return svk::set_error(st, m); }

}  // namespace

namespace svk {

sv_status plan_create(sv_state s, const sv_gate *gates, size_t n_gates, sv_plan *out, std::string *err,
                      bool relabel)
{
    if (s->n < 4) {
        *err = "planned circuits need at least 4 qubits";
        return SV_EINVAL;
    }
    TileGeom geo = geometry(s->n, s->dt, 4, s);
    std::vector<Item> items;
    items.reserve(n_gates);
    for (size_t i = 0; i < n_gates; ++i) items.push_back(classify(gates[i], int(i)));
    bool ok = true;
    const std::vector<PPass> passes = plan_passes_geo(s->n, geo, items, &ok, relabel);
    if (!ok) {
        *err = "planner could not place every gate with this tile geometry";
        return SV_EUNSUPPORTED;
    }
    Flat f = flatten(s->n, geo, passes);
    if (!f.ok) {
        *err = "planner left a diagonal pair term outside the tile";
        return SV_EUNSUPPORTED;
    }
    const bool c64 = s->dt == SV_C64;
    const size_t tab_bytes = 512 * (c64 ? sizeof(float2) : sizeof(double2));
    const size_t off_ops = align_up(f.groups.size() * sizeof(TileGroup), 256);
    const size_t off_dtab = align_up(off_ops + f.ops.size() * sizeof(TileOp), 256);
    const size_t off_tab = align_up(off_dtab + f.dtab.size() * sizeof(uint64_t), 256);
    const size_t total = off_tab + tab_bytes;
    std::vector<char> h(total);
    std::memcpy(h.data(), f.groups.data(), f.groups.size() * sizeof(TileGroup));
    std::memcpy(h.data() + off_ops, f.ops.data(), f.ops.size() * sizeof(TileOp));
    std::memcpy(h.data() + off_dtab, f.dtab.data(), f.dtab.size() * sizeof(uint64_t));
    if (c64) fill_phase_table(reinterpret_cast<float2 *>(h.data() + off_tab));
    else fill_phase_table(reinterpret_cast<double2 *>(h.data() + off_tab));
    static std::atomic<uint64_t> next_serial{1};
    sv_plan p = new (std::nothrow) sv_plan_s;
    if (!p) { *err = "host allocation failed"; return SV_ENOMEM; }
    p->serial = next_serial.fetch_add(1);
    hipError_t e = hipMalloc(&p->dev, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        *err = "device allocation of the plan failed";
        return SV_ENOMEM;
    }
    // Synchronous upload: plans are built once, outside the hot loop.
    e = hipMemcpy(p->dev, h.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        delete p;
        *err = hipGetErrorString(e);
        return SV_EDEVICE;
    }
    char *d = static_cast<char *>(p->dev);
    for (TileArgs a : f.args) {
        a.psi = s->psi;
        a.groups = reinterpret_cast<const TileGroup *>(d);
        a.ops = reinterpret_cast<const TileOp *>(d + off_ops);
        a.dtab = reinterpret_cast<const uint64_t *>(d + off_dtab);
        a.phase_tab = d + off_tab;
        p->passes.push_back(a);
    }
    p->flops = f.flops;
    p->st = s;
    p->n = s->n;
    p->dt = s->dt;
    *out = p;
    return SV_OK;
}

}  // namespace svk

extern "C" {

sv_status sv_plan_destroy(sv_plan p)
{
    if (!p) return SV_OK;
    if (p->dev) (void)hipFree(p->dev);   // waits for work that may still read it
    delete p;
    return SV_OK;
}

sv_status sv_plan_passes(sv_plan p, int32_t *n_passes)
{
    if (!p || !n_passes) return berr(SV_EINVAL, "null argument");
    *n_passes = int32_t(p->passes.size());
    return SV_OK;
}

sv_status sv_run_plan(sv_plan p, int32_t first_pass, int32_t count)
{
    if (!p) return berr(SV_EINVAL, "null plan");
    if (first_pass < 0 || count < 0 || size_t(first_pass) + size_t(count) > p->passes.size())
        return berr(SV_EINVAL, "pass range outside the plan");
    sv_state s = p->st;
    const double bytes = 2.0 * std::ldexp(1.0, s->n) * svk::elem_bytes(s->dt);
    for (int32_t i = first_pass; i < first_pass + count; ++i) {
        const int tok = svk::prof_begin(s);
        hipError_t e = svk::launch_tile(p->passes[i], 4, s->dt == SV_C64, s->stream);
        svk::prof_end(s, tok, svk::KC_TILE, bytes, p->flops[i]);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("tile launch: ") + hipGetErrorString(e));
    }
    return SV_OK;
}

sv_status sv_batch_create(sv_dtype dtype, void *hip_stream, sv_batch *out)
{
    if (!out) return berr(SV_EINVAL, "null output pointer");
    if (dtype != SV_C64 && dtype != SV_C128) return berr(SV_EINVAL, "unknown dtype");
    sv_batch b = new (std::nothrow) sv_batch_s;
    if (!b) return berr(SV_ENOMEM, "host allocation failed");
    b->dt = dtype;
    b->stream = static_cast<hipStream_t>(hip_stream);
    // Complex64 batch kernels hold three work-groups per CU, complex128 ones
    // two (the tuned configurations of the 512-circuit batch: 3x4 for complex64).
    if (dtype == SV_C64) {
        b->blocks_per_cu = 3;
        b->tiles_per_task = 4;
    }
    if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return berr(SV_EDEVICE, "event creation failed");
    }
    *out = b;
    return SV_OK;
}

sv_status sv_batch_destroy(sv_batch b)
{
    if (!b) return SV_OK;
    (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->side) {
        (void)hipStreamSynchronize(b->side);
        (void)hipStreamDestroy(b->side);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->solo) {
        (void)hipStreamSynchronize(b->solo);
        (void)hipStreamDestroy(b->solo);
    }
    if (b->sfork) (void)hipEventDestroy(b->sfork);
    if (b->sjoin) (void)hipEventDestroy(b->sjoin);
    if (b->work.dev) (void)hipFree(b->work.dev);
    if (b->gimg.dev) (void)hipFree(b->gimg.dev);
    if (b->host) (void)hipHostFree(b->host);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
    return SV_OK;
}

sv_status sv_batch_persist(sv_batch b, int32_t max_tiles)
{
    if (!b) return berr(SV_EINVAL, "null batch");
    if (max_tiles < 0 || max_tiles > (1 << 20)) return berr(SV_EINVAL, "max_tiles out of range");
    b->persist_tiles = max_tiles;
    return SV_OK;
}

sv_status sv_batch_solo(sv_batch b, int32_t min_tiles)
{
    if (!b) return berr(SV_EINVAL, "null batch");
    if (min_tiles < 0) return berr(SV_EINVAL, "min_tiles is negative");
    b->solo_tiles = min_tiles;
    return SV_OK;
}

sv_status sv_batch_config(sv_batch b, int32_t blocks_per_cu, int32_t tiles_per_task)
{
    if (!b) return berr(SV_EINVAL, "null batch");
    if (blocks_per_cu < 1 || blocks_per_cu > 8) return berr(SV_EINVAL, "blocks_per_cu not in [1, 8]");
    if (tiles_per_task < 1 || tiles_per_task > 4096) return berr(SV_EINVAL, "tiles_per_task not in [1, 4096]");
    if (b->blocks_per_cu != blocks_per_cu || b->tiles_per_task != uint32_t(tiles_per_task)) {
        b->blocks_per_cu = blocks_per_cu;
        b->tiles_per_task = uint32_t(tiles_per_task);
        b->gkey.clear();   // a captured graph used the old configuration
    }
    return SV_OK;
}

namespace {

// Builds the level-ordered task list of a batch into `img` (device buffers
// grown as needed) and queues its upload on `st` through pinned staging.
int device_cus()
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

sv_status prepare_batch(sv_batch b, BatchImage &img, const sv_plan *plans,
                        const std::vector<int32_t> &first, const std::vector<int32_t> &cnt,
                        hipStream_t st)
{
    using namespace svk;
    const size_t count = first.size();
    std::vector<TileArgs> passes;
    std::vector<size_t> pass0(count);
    for (size_t i = 0; i < count; ++i) {
        pass0[i] = passes.size();
        for (int32_t k = 0; k < cnt[i]; ++k) passes.push_back(plans[i]->passes[first[i] + k]);
    }
    // Levels by list scheduling, least remaining work first: a level takes the
    // next pass of circuits in order of remaining work (passes left times
    // amplitudes) until it holds about one round of tasks for every resident
    // work-group, so each launch fills the GPU while small circuits finish
    // early instead of waiting for every big circuit's pass at each level.
    // A circuit has at most one pass per level, so its passes stay in order.
    // (512-circuit batch, rounds per level 0.5 / 0.75 / 1 / 1.5 / 2 / 4:
    // makespan 915 / 827 / 790 / 815 / 824 / 842 ms, p50 9.8 / 9.8 / 10.0 /
    // 12.1 / 13.0 / 17.1 ms, p99 847 / 776 / 730 / 703 / 712 / 730 ms.)
    // Levels alone, with no persistent launch or third stream to fill the
    // gaps between them, take two rounds (makespan 882 ms against 980 ms).
    std::vector<BatchTask> tasks;
    img.level0.clear();
    img.task_circ.clear();
    std::vector<uint64_t> amps(count, 0);
    for (size_t i = 0; i < count; ++i)
        if (cnt[i] > 0) {
            const TileArgs &p0 = passes[pass0[i]];
            amps[i] = p0.ntiles << p0.L;
        }
    const uint64_t rounds = (b->persist_tiles > 0 || b->solo_tiles > 0) ? 1 : 2;
    const uint64_t cap = uint64_t(device_cus()) * uint64_t(std::max(1, b->blocks_per_cu)) *
                         uint64_t(b->tiles_per_task) * rounds * (uint64_t(1) << 12);
    std::vector<int32_t> done(count, 0);
    // Small circuits go whole to the persistent launch, least work first.
    std::vector<PersistCircuit> circs;
    img.pcirc.clear();
    if (b->persist_tiles > 0) {
        std::vector<size_t> small;
        for (size_t i = 0; i < count; ++i)
            if (cnt[i] > 0 && passes[pass0[i]].ntiles <= uint64_t(b->persist_tiles)) small.push_back(i);
        std::stable_sort(small.begin(), small.end(), [&](size_t x, size_t y) {
            return uint64_t(cnt[x]) * amps[x] < uint64_t(cnt[y]) * amps[y];
        });
        for (size_t i : small) {
            circs.push_back(PersistCircuit{int32_t(pass0[i]), cnt[i]});
            img.pcirc.push_back(int32_t(i));
            done[i] = cnt[i];
        }
    }
    // Large circuits run pass by pass beside the levels, least work first.
    img.scirc.clear();
    img.sfirst.clear();
    img.scount.clear();
    img.spasses.clear();
    if (b->solo_tiles > 0) {
        std::vector<size_t> large;
        for (size_t i = 0; i < count; ++i)
            if (done[i] < cnt[i] && passes[pass0[i]].ntiles >= uint64_t(b->solo_tiles)) large.push_back(i);
        std::stable_sort(large.begin(), large.end(), [&](size_t x, size_t y) {
            return uint64_t(cnt[x]) * amps[x] < uint64_t(cnt[y]) * amps[y];
        });
        for (size_t i : large) {
            img.scirc.push_back(int32_t(i));
            img.sfirst.push_back(int32_t(img.spasses.size()));
            img.scount.push_back(cnt[i]);
            for (int32_t k = 0; k < cnt[i]; ++k) img.spasses.push_back(passes[pass0[i] + k]);
            done[i] = cnt[i];
        }
    }
    std::vector<size_t> order;
    order.reserve(count);
    for (;;) {
        order.clear();
        for (size_t i = 0; i < count; ++i)
            if (done[i] < cnt[i]) order.push_back(i);
        if (order.empty()) break;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            return uint64_t(cnt[x] - done[x]) * amps[x] < uint64_t(cnt[y] - done[y]) * amps[y];
        });
        img.level0.push_back(uint32_t(tasks.size()));
        uint64_t level_amps = 0;
        for (size_t i : order) {
            if (level_amps >= cap) break;
            const int32_t pi = int32_t(pass0[i]) + done[i];
            const uint64_t nt = passes[pi].ntiles;
            for (uint64_t t0 = 0; t0 < nt; t0 += b->tiles_per_task) {
                BatchTask t;
                t.pass = pi;
                t.circ = int32_t(i);
                t.tile0 = uint32_t(t0);
                t.ntiles = uint32_t(std::min<uint64_t>(b->tiles_per_task, nt - t0));
                tasks.push_back(t);
                img.task_circ.push_back(int32_t(i));
            }
            level_amps += amps[i];
            ++done[i];
        }
    }
    img.level0.push_back(uint32_t(tasks.size()));
    img.count = count;
    img.off_pass = align_up(tasks.size() * sizeof(BatchTask), 256);
    img.off_circ = align_up(img.off_pass + passes.size() * sizeof(TileArgs), 256);
    img.off_start = align_up(img.off_circ + circs.size() * sizeof(PersistCircuit), 256);
    img.off_end = align_up(img.off_start + tasks.size() * sizeof(uint64_t), 256);
    img.off_pstart = align_up(img.off_end + tasks.size() * sizeof(uint64_t), 256);
    img.off_pend = align_up(img.off_pstart + circs.size() * sizeof(uint64_t), 256);
    img.off_sstart = align_up(img.off_pend + circs.size() * sizeof(uint64_t), 256);
    img.off_send = align_up(img.off_sstart + img.scirc.size() * sizeof(uint64_t), 256);
    const size_t total = align_up(img.off_send + img.scirc.size() * sizeof(uint64_t), 256);
    const size_t upload = img.off_start;
    hipError_t e = hipEventSynchronize(b->staged);   // staging free again
    if (e != hipSuccess) return berr(SV_EDEVICE, hipGetErrorString(e));
    if (b->host_cap < upload) {
        if (b->host) (void)hipHostFree(b->host);
        b->host = nullptr;
        b->host_cap = 0;
        if (hipHostMalloc(&b->host, upload, 0) != hipSuccess) return berr(SV_ENOMEM, "pinned staging failed");
        b->host_cap = upload;
    }
    if (img.cap < total) {
        if (img.dev) (void)hipFree(img.dev);   // waits for work that may use it
        img.dev = nullptr;
        img.cap = 0;
        if (hipMalloc(&img.dev, total) != hipSuccess) {
            (void)hipGetLastError();
            return berr(SV_ENOMEM, "batch workspace allocation failed");
        }
        img.cap = total;
    }
    char *h = static_cast<char *>(b->host);
    std::memcpy(h, tasks.data(), tasks.size() * sizeof(BatchTask));
    std::memcpy(h + img.off_pass, passes.data(), passes.size() * sizeof(TileArgs));
    std::memcpy(h + img.off_circ, circs.data(), circs.size() * sizeof(PersistCircuit));
    e = hipMemcpyAsync(img.dev, h, upload, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(b->staged, st);
    if (e != hipSuccess) return berr(SV_EDEVICE, hipGetErrorString(e));
    return SV_OK;
}

// Device clock (the one the level tasks stamp) at this point of the stream.
__global__ void k_stamp(uint64_t *slot)
{
    if (threadIdx.x == 0) *slot = wall_clock64();
}

// Queues the persistent launch (if any circuit takes it) on the side stream,
// forked from `st` after the upload and joined back at the end, and one launch
// per level of `img` on `st`: the two work on disjoint states, so the short
// circuits run beside the first levels of the long ones. Both streams have the
// default priority; under capture the side stream joins the graph through the
// fork event.
sv_status launch_levels(sv_batch b, const BatchImage &img, hipStream_t st)
{
    using namespace svk;
    char *d = static_cast<char *>(img.dev);
    const bool side = !img.pcirc.empty();
    if (side) {
        if (!b->side || !b->fork || !b->join) return berr(SV_EDEVICE, "side stream not set up");
        hipError_t e = hipEventRecord(b->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->fork, 0);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("side stream: ") + hipGetErrorString(e));
    }
    if (side) {
        PersistArgs p{};
        p.circs = reinterpret_cast<const PersistCircuit *>(d + img.off_circ);
        p.passes = reinterpret_cast<const TileArgs *>(d + img.off_pass);
        p.t_start = reinterpret_cast<uint64_t *>(d + img.off_pstart);
        p.t_end = reinterpret_cast<uint64_t *>(d + img.off_pend);
        p.count = uint32_t(img.pcirc.size());
        hipError_t e = launch_persist(p, b->dt == SV_C64, b->blocks_per_cu, b->side);
        if (e == hipSuccess) e = hipEventRecord(b->join, b->side);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("persistent launch: ") + hipGetErrorString(e));
    }
    // Large circuits go to the third stream, forked from `st` after the first
    // sixteenth of the levels: the short circuits of those levels finish
    // before the large passes share the device (p50 34 -> 20 ms on the
    // 512-circuit batch, makespan +0.4 %).
    const bool solo = !img.scirc.empty();
    auto queue_large = [&]() -> sv_status {
        if (!b->solo || !b->sfork || !b->sjoin) return berr(SV_EDEVICE, "third stream not set up");
        hipError_t e = hipEventRecord(b->sfork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->solo, b->sfork, 0);
        uint64_t *t0 = reinterpret_cast<uint64_t *>(d + img.off_sstart);
        uint64_t *t1 = reinterpret_cast<uint64_t *>(d + img.off_send);
        for (size_t k = 0; k < img.scirc.size() && e == hipSuccess; ++k) {
            hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, b->solo, t0 + k);
            e = hipGetLastError();
            for (int32_t j = 0; j < img.scount[k] && e == hipSuccess; ++j)
                e = launch_tile(img.spasses[size_t(img.sfirst[k] + j)], 4, b->dt == SV_C64, b->solo);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, b->solo, t1 + k);
                e = hipGetLastError();
            }
        }
        if (e == hipSuccess) e = hipEventRecord(b->sjoin, b->solo);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("large circuits: ") + hipGetErrorString(e));
        return SV_OK;
    };
    BatchArgs a{};
    a.tasks = reinterpret_cast<const BatchTask *>(d);
    a.passes = reinterpret_cast<const TileArgs *>(d + img.off_pass);
    a.t_start = reinterpret_cast<uint64_t *>(d + img.off_start);
    a.t_end = reinterpret_cast<uint64_t *>(d + img.off_end);
    const size_t nlev = img.level0.size() - 1;
    const size_t fork_at = nlev / 16;
    if (solo && fork_at == 0)
        if (sv_status r = queue_large()) return r;
    for (size_t lev = 0; lev < nlev; ++lev) {
        a.task0 = img.level0[lev];
        a.task_end = img.level0[lev + 1];
        hipError_t e = launch_level(a, b->dt == SV_C64, b->blocks_per_cu, st);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("level launch: ") + hipGetErrorString(e));
        if (solo && fork_at == lev + 1)
            if (sv_status r = queue_large()) return r;
    }
    if (side) {
        hipError_t e = hipStreamWaitEvent(st, b->join, 0);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("side join: ") + hipGetErrorString(e));
    }
    if (solo) {
        hipError_t e = hipStreamWaitEvent(st, b->sjoin, 0);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("third stream join: ") + hipGetErrorString(e));
    }
    return SV_OK;
}

}  // namespace

sv_status sv_batch_run(sv_batch b, const sv_plan *plans, const int32_t *first_pass,
                       const int32_t *pass_count, size_t count, uint32_t flags)
{
    if (!b) return berr(SV_EINVAL, "null batch");
    if (flags & ~SV_GRAPH) return berr(SV_EINVAL, "unknown batch flags");
    if (count == 0) return SV_OK;
    if (!plans) return berr(SV_EINVAL, "null plan array");
    if (count > (1u << 20)) return berr(SV_EINVAL, "too many circuits in one batch");
    std::vector<int32_t> first(count), cnt(count);
    std::vector<uintptr_t> key;
    key.reserve(3 * count + 2);
    key.push_back(uintptr_t(b->blocks_per_cu));
    key.push_back(uintptr_t(b->tiles_per_task));
    key.push_back(uintptr_t(b->persist_tiles));
    key.push_back(uintptr_t(b->solo_tiles));
    for (size_t i = 0; i < count; ++i) {
        const sv_plan p = plans[i];
        if (!p) return berr(SV_EINVAL, "null plan in batch");
        if (p->dt != b->dt) return berr(SV_EINVAL, "plan dtype differs from the batch dtype");
        first[i] = first_pass ? first_pass[i] : 0;
        cnt[i] = pass_count ? pass_count[i] : int32_t(p->passes.size()) - first[i];
        if (first[i] < 0 || cnt[i] < 0 || size_t(first[i]) + size_t(cnt[i]) > p->passes.size())
            return berr(SV_EINVAL, "pass range outside a plan");
        for (size_t j = 0; j < i; ++j)
            if (plans[j]->st == p->st) return berr(SV_EINVAL, "two plans of one state in a batch");
        key.push_back(uintptr_t(p->serial));
        key.push_back(uintptr_t(first[i]));
        key.push_back(uintptr_t(cnt[i]));
    }
    if (b->persist_tiles > 0) {   // the side stream and its events exist before any capture
        hipError_t e = hipSuccess;
        if (!b->side) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess && !b->fork) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess && !b->join) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("side stream: ") + hipGetErrorString(e));
    }
    if (b->solo_tiles > 0) {      // so do the third stream and its events
        hipError_t e = hipSuccess;
        if (!b->solo) e = hipStreamCreateWithFlags(&b->solo, hipStreamNonBlocking);
        if (e == hipSuccess && !b->sfork) e = hipEventCreateWithFlags(&b->sfork, hipEventDisableTiming);
        if (e == hipSuccess && !b->sjoin) e = hipEventCreateWithFlags(&b->sjoin, hipEventDisableTiming);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("third stream: ") + hipGetErrorString(e));
    }
    if (!(flags & SV_GRAPH)) {
        if (sv_status st = prepare_batch(b, b->work, plans, first, cnt, b->stream)) return st;
        if (sv_status st = launch_levels(b, b->work, b->stream)) return st;
        b->last = &b->work;
        return SV_OK;
    }
    // SV_GRAPH: capture the level launches once per content, then replay.
    if (!b->gexec || b->gkey != key) {
        if (b->gexec) {
            (void)hipStreamSynchronize(b->stream);
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
        b->gkey.clear();
        if (!b->capture && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
            return berr(SV_EDEVICE, "capture stream creation failed");
        if (sv_status st = prepare_batch(b, b->gimg, plans, first, cnt, b->capture)) return st;
        hipError_t e = hipStreamSynchronize(b->capture);   // buffers uploaded before capture
        if (e != hipSuccess) return berr(SV_EDEVICE, hipGetErrorString(e));
        e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("begin capture: ") + hipGetErrorString(e));
        sv_status st = launch_levels(b, b->gimg, b->capture);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(b->capture, &graph);
        if (st != SV_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return berr(SV_EDEVICE, std::string("end capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            return berr(SV_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        b->gkey = key;
    }
    hipError_t e = hipGraphLaunch(b->gexec, b->stream);
    if (e != hipSuccess) return berr(SV_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    b->last = &b->gimg;
    return SV_OK;
}

sv_status sv_batch_times(sv_batch b, double *start_ms, double *end_ms, size_t count)
{
    if (!b) return berr(SV_EINVAL, "null batch");
    const BatchImage *img = b->last;
    if (!img || count != img->count) return berr(SV_EINVAL, "count differs from the last run");
    const size_t nt = img->task_circ.size(), np = img->pcirc.size(), ns = img->scirc.size();
    // Task clocks, the persistent circuits' clocks and the large circuits'
    // stamps, as one list.
    std::vector<uint64_t> t0(nt + np + ns), t1(nt + np + ns);
    std::vector<int32_t> circ_of(img->task_circ);
    circ_of.insert(circ_of.end(), img->pcirc.begin(), img->pcirc.end());
    circ_of.insert(circ_of.end(), img->scirc.begin(), img->scirc.end());
    hipError_t e = hipSuccess;
    char *dev = static_cast<char *>(img->dev);
    if (nt) {
        e = hipMemcpyAsync(t0.data(), dev + img->off_start, nt * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t1.data(), dev + img->off_end, nt * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, b->stream);
    }
    if (np && e == hipSuccess) {
        e = hipMemcpyAsync(t0.data() + nt, dev + img->off_pstart, np * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t1.data() + nt, dev + img->off_pend, np * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, b->stream);
    }
    if (ns && e == hipSuccess) {
        e = hipMemcpyAsync(t0.data() + nt + np, dev + img->off_sstart, ns * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t1.data() + nt + np, dev + img->off_send, ns * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return berr(SV_EDEVICE, hipGetErrorString(e));
    const int khz = svk::wall_clock_khz();
    uint64_t origin = ~uint64_t(0);
    for (size_t k = 0; k < nt + np + ns; ++k) origin = std::min(origin, t0[k]);
    std::vector<uint64_t> first(count, ~uint64_t(0)), last(count, 0);
    for (size_t k = 0; k < nt + np + ns; ++k) {
        const int32_t c = circ_of[k];
        first[c] = std::min(first[c], t0[k]);
        last[c] = std::max(last[c], t1[k]);
    }
    for (size_t i = 0; i < count; ++i) {
        const bool none = first[i] == ~uint64_t(0);   // no passes in the run
        if (start_ms) start_ms[i] = none ? 0.0 : double(first[i] - origin) / khz;
        if (end_ms) end_ms[i] = none ? 0.0 : double(last[i] - origin) / khz;
    }
    return SV_OK;
}

}  // extern "C"
