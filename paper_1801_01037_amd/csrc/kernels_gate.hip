// Per-gate kernels: basis-state init, the 2x2 pair update (plain, controlled,
// exchange-only) and diagonal runs.
//
// The pair update is the stride rule of State Vector Partitioning: for a gate
// on qubit t every pair (i0, i0 + 2^t) with bit t of i0 clear becomes
// (q11 a + q12 b, q21 a + q22 b); a control c restricts it to indices with bit
// c set (caption of Algorithm 1), several controls (a Toffoli gate has two) to
// indices with all of them set. Instead of the paper's two nested loops, a
// flat work index is expanded by inserting the fixed bits (target = 0,
// controls = 1) that select whole 128-byte lines, so consecutive lanes touch
// consecutive 16-byte chunks and every line is read and written whole: when
// the two halves of a pair lie in different lines they form two coalesced
// streams; when they lie in one line, lanes holding the two chunks swap them
// by a cross-lane permute; controls inside a line are tested per amplitude.
#include <type_traits>

#include "sv_internal.h"

namespace svk {
namespace {

constexpr int kBlock = 256;

// x with bit value v inserted at position p (bits at and above p move up).
__device__ __forceinline__ uint64_t insert_bit(uint64_t x, int p, uint64_t v)
{
    const uint64_t lo = x & ((uint64_t(1) << p) - 1);
    return ((x >> p) << (p + 1)) | (v << p) | lo;
}

template <typename R>
struct CMat {
    R r11, i11, r12, i12, r21, i21, r22, i22;
};

template <typename R>
CMat<R> to_cmat(const Mat2 &m)
{
    return CMat<R>{R(m.q[0]), R(m.q[1]), R(m.q[2]), R(m.q[3]),
                   R(m.q[4]), R(m.q[5]), R(m.q[6]), R(m.q[7])};
}

// (a, b) <- (q11 a + q12 b, q21 a + q22 b) in precision R.
template <typename R>
__device__ __forceinline__ void pair_update(R &ar, R &ai, R &br, R &bi, const CMat<R> &m)
{
    const R nar = m.r11 * ar - m.i11 * ai + m.r12 * br - m.i12 * bi;
    const R nai = m.r11 * ai + m.i11 * ar + m.r12 * bi + m.i12 * br;
    const R nbr = m.r21 * ar - m.i21 * ai + m.r22 * br - m.i22 * bi;
    const R nbi = m.r21 * ai + m.i21 * ar + m.r22 * bi + m.i22 * br;
    ar = nar; ai = nai; br = nbr; bi = nbi;
}

// Where the two amplitudes of a pair sit relative to 16-byte chunks and
// 128-byte lines (8 chunks).
enum Layout {
    kSplit = 0,    // a and b in different lines, 2^t apart: two coalesced streams
    kLane = 1,     // a and b in chunks of one wave's 64 consecutive chunks: lanes exchange
    kInChunk = 2,  // complex64, t = 0: one chunk holds (a, b)
};

template <typename R>
struct PairArgs {
    void *psi;
    uint64_t items;       // work items: chunk pairs (kSplit) or chunks
    uint64_t tstride;     // 2^t in amplitudes
    uint64_t clow;        // controls below the line: tested per amplitude
    int nins;             // fixed index bits to insert, ascending positions
    uint64_t vals;        // bit k: the value inserted at pos[k]
    uint32_t xcd_span;    // nonzero: work-groups per XCD, see xcd_block
    CMat<R> m;
    uint8_t pos[64];
};


// Chunk index of work item `item`: the fixed bits (all at or above the line)
// inserted into item * E, over E.
template <uint64_t E, typename A>
__device__ __forceinline__ uint64_t chunk_of(uint64_t item, const A &a)
{
    uint64_t x = item * E;
    for (int k = 0; k < a.nins; ++k) x = insert_bit(x, a.pos[k], (a.vals >> k) & 1u);
    return x / E;
}

// (a, b) of one pair, updated when its index i has every low control set.
template <typename R, bool SWAP>
__device__ __forceinline__ void pair_if(R &ar, R &ai, R &br, R &bi, uint64_t i,
                                        const PairArgs<R> &a)
{
    if ((i & a.clow) != a.clow) return;
    if constexpr (SWAP) {
        R t = ar; ar = br; br = t;
        t = ai; ai = bi; bi = t;
    } else {
        pair_update<R>(ar, ai, br, bi, a.m);
    }
}

// One output of a pair whose halves sit in two lanes: this lane holds `own`
// (the half with bit t = hi) and receives the other half `oth`.
template <typename R, bool SWAP>
__device__ __forceinline__ void half_if(R &r, R &i, R orr, R oi, bool hi, uint64_t idx,
                                        const PairArgs<R> &a)
{
    if ((idx & a.clow) != a.clow) return;
    if constexpr (SWAP) {
        r = orr; i = oi;
    } else if (!hi) {
        const R nr = a.m.r11 * r - a.m.i11 * i + a.m.r12 * orr - a.m.i12 * oi;
        const R ni = a.m.r11 * i + a.m.i11 * r + a.m.r12 * oi + a.m.i12 * orr;
        r = nr; i = ni;
    } else {
        const R nr = a.m.r21 * orr - a.m.i21 * oi + a.m.r22 * r - a.m.i22 * i;
        const R ni = a.m.r21 * oi + a.m.i21 * orr + a.m.r22 * i + a.m.i22 * r;
        r = nr; i = ni;
    }
}

// U work items per thread: items first + u * kBlock (a block's items are
// kBlock-strided per thread), or with RUNS the U items of a thread are
// neighbours in its wave's run of 64 U items, so each wave reads each half of
// its pairs in runs of U KiB.
template <bool C64, int LAYOUT, bool SWAP, bool NT, int U, bool RUNS = false>
__global__ __launch_bounds__(kBlock) void k_pair(PairArgs<std::conditional_t<C64, float, double>> a)
{
    using R = std::conditional_t<C64, float, double>;
    using V = std::conditional_t<C64, float4, double2>;   // one 16-byte chunk
    constexpr uint64_t E = C64 ? 2 : 1;                   // amplitudes per chunk
    V *p = static_cast<V *>(a.psi);
    const uint64_t first = uint64_t(xcd_block(blockIdx.x, a.xcd_span)) * (kBlock * U) + threadIdx.x;

    if constexpr (LAYOUT == kLane) {
        // Consecutive lanes hold consecutive chunks (the bits inserted into
        // the work index all lie above the target), so the partner chunk,
        // 2^t / E < 64 chunks away, is in lane lane ^ (2^t / E) of the same
        // wave. Every lane takes part in the exchange; lanes past the end
        // carry zeros and store nothing.
        const int d = int(a.tstride / E);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t item = first + uint64_t(u) * kBlock;
            const bool live = item < a.items;
            const uint64_t c = chunk_of<E>(item, a);
            V v;
            if (live) v = ld16<NT>(&p[c]);
            else if constexpr (C64) v = make_float4(0.f, 0.f, 0.f, 0.f);
            else v = make_double2(0.0, 0.0);
            V o;
            o.x = __shfl_xor(v.x, d);
            o.y = __shfl_xor(v.y, d);
            if constexpr (C64) {
                o.z = __shfl_xor(v.z, d);
                o.w = __shfl_xor(v.w, d);
            }
            const bool hi = (c & uint64_t(d)) != 0;
            if constexpr (C64) {
                half_if<R, SWAP>(v.x, v.y, o.x, o.y, hi, c * E, a);
                half_if<R, SWAP>(v.z, v.w, o.z, o.w, hi, c * E + 1, a);
            } else {
                half_if<R, SWAP>(v.x, v.y, o.x, o.y, hi, c, a);
            }
            if (live) st16<NT>(&p[c], v);
        }
        return;
    } else {
        V va[U], vb[U];
        uint64_t ca[U];
        // the item of this thread's u-th chunk
        auto item_of = [&](int u) {
            if constexpr (RUNS)
                return uint64_t(xcd_block(blockIdx.x, a.xcd_span)) * (kBlock * U) +
                       uint64_t(threadIdx.x / 64) * (64 * U) + uint64_t(u) * 64 + (threadIdx.x % 64);
            else
                return first + uint64_t(u) * kBlock;
        };
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t item = item_of(u);
            ca[u] = chunk_of<E>(item, a);
            if (item < a.items) {
                va[u] = ld16<NT>(&p[ca[u]]);
                if (LAYOUT == kSplit) vb[u] = ld16<NT>(&p[ca[u] + a.tstride / E]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t item = item_of(u);
            if (item >= a.items) continue;
            const uint64_t i0 = ca[u] * E;
            if constexpr (LAYOUT == kInChunk) {
                pair_if<R, SWAP>(va[u].x, va[u].y, va[u].z, va[u].w, i0, a);
            } else if constexpr (C64) {
                pair_if<R, SWAP>(va[u].x, va[u].y, vb[u].x, vb[u].y, i0, a);
                pair_if<R, SWAP>(va[u].z, va[u].w, vb[u].z, vb[u].w, i0 + 1, a);
            } else {
                pair_if<R, SWAP>(va[u].x, va[u].y, vb[u].x, vb[u].y, i0, a);
            }
            st16<NT>(&p[ca[u]], va[u]);
            if (LAYOUT == kSplit) st16<NT>(&p[ca[u] + a.tstride / E], vb[u]);
        }
    }
}

template <bool C64>
struct InitArgs {
    void *psi;
    uint64_t chunks;
    uint64_t basis;
};

template <bool C64>
__global__ __launch_bounds__(kBlock) void k_init(InitArgs<C64> a)
{
    using V = std::conditional_t<C64, float4, double2>;
    constexpr uint64_t E = C64 ? 2 : 1;
    V *p = static_cast<V *>(a.psi);
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    // Each XCD writes one contiguous eighth of every stride (complex64 5.2 ->
    // 5.9 TB/s, complex128 5.4 -> 5.8 TB/s).
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0);
    for (uint64_t c = uint64_t(b) * kBlock + threadIdx.x; c < a.chunks; c += stride) {
        V v;
        if constexpr (C64) {
            v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c == a.basis / E) {
                if (a.basis % E == 0) v.x = 1.f; else v.z = 1.f;
            }
        } else {
            v = make_double2(c == a.basis ? 1.0 : 0.0, 0.0);
        }
        p[c] = v;
    }
}

struct DiagArgs {
    void *psi;
    uint64_t items;       // chunks to visit
    int nins;             // bits at or above the line fixed to 1 in every visited index (ascending)
    int pos[4];
    int count;
    uint32_t xcd_span;    // nonzero: work-groups per XCD, see xcd_block
    DiagTerm t[kMaxDiagTerms];
};

// e^{2 pi i T / 2^64} in FP64: T read as a signed fraction of a half turn.
__device__ __forceinline__ void turn_phase(uint64_t T, double &c, double &s)
{
    const double f = double(int64_t(T)) * 0x1p-63;
    sincospi(f, &s, &c);
}

__device__ __forceinline__ uint64_t turn_of(uint64_t i, const DiagArgs &a)
{
    uint64_t T = 0;
    for (int k = 0; k < a.count; ++k)
        T += ((i & a.t[k].mask) == a.t[k].val) ? a.t[k].turn : 0;
    return T;
}

// Chunks whose phase is 1 are written back only when streaming (NT), so
// that every line goes out whole.
template <bool C64, bool NT, int U>
__global__ __launch_bounds__(kBlock) void k_diag(DiagArgs a)
{
    using V = std::conditional_t<C64, float4, double2>;
    constexpr uint64_t E = C64 ? 2 : 1;
    V *p = static_cast<V *>(a.psi);
    const uint64_t first = uint64_t(xcd_block(blockIdx.x, a.xcd_span)) * (kBlock * U) + threadIdx.x;
    V v[U];
    uint64_t ci[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        uint64_t x = item * E;
        for (int k = 0; k < a.nins; ++k) x = insert_bit(x, a.pos[k], 1);
        ci[u] = x / E;
        if (item < a.items) v[u] = ld16<NT>(&p[ci[u]]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        if (item >= a.items) continue;
        const uint64_t i0 = ci[u] * E;
        if constexpr (C64) {
            const uint64_t T0 = turn_of(i0, a), T1 = turn_of(i0 + 1, a);
            if (!NT && (T0 | T1) == 0) continue;
            double c, s;
            if (T0) {
                turn_phase(T0, c, s);
                const float fc = float(c), fs = float(s);
                const float re = v[u].x * fc - v[u].y * fs;
                const float im = v[u].x * fs + v[u].y * fc;
                v[u].x = re; v[u].y = im;
            }
            if (T1) {
                turn_phase(T1, c, s);
                const float fc = float(c), fs = float(s);
                const float re = v[u].z * fc - v[u].w * fs;
                const float im = v[u].z * fs + v[u].w * fc;
                v[u].z = re; v[u].w = im;
            }
        } else {
            const uint64_t T = turn_of(i0, a);
            if (!NT && T == 0) continue;
            if (T) {
                double c, s;
                turn_phase(T, c, s);
                const double re = v[u].x * c - v[u].y * s;
                const double im = v[u].x * s + v[u].y * c;
                v[u].x = re; v[u].y = im;
            }
        }
        st16<NT>(&p[ci[u]], v[u]);
    }
}

constexpr int kDiagU = 2;

// A launch holds fewer than 2^32 work-items along x; per-gate launches keep
// to 2^31 and give each thread four items when a state has more.
constexpr uint64_t kMaxLaunchItems = uint64_t(1) << 31;

inline unsigned grid_for(uint64_t items, int per_block)
{
    return unsigned((items + per_block - 1) / per_block);
}


template <bool C64, int LAYOUT, bool SWAP, bool NT>
hipError_t launch_pair_u(PairArgs<std::conditional_t<C64, float, double>> a, hipStream_t st)
{
    // One pair per thread; four when the state has more pairs than a launch
    // holds work-items. Grids that split evenly over the XCDs get the
    // XCD-contiguous order (30-qubit 1q median over targets 5.98 -> 6.20 TB/s).
    // Pairs whose halves lie 256 MiB or 4 GiB or more apart take two
    // neighbouring chunks per thread, read in 2 KiB runs per wave. Both
    // halves of a pair then fall on the same memory banks (the slow strides
    // repeat every four address bits from 16 MiB); at these strides the
    // longer runs were measured faster at 30 qubits: complex128 targets 24
    // 5.60 -> 5.75 TB/s, 28 5.55 -> 5.84, 29 5.78 -> 5.85; complex64 targets
    // 25 5.63 -> 5.76, 29 5.56 -> 5.80. At 16 MiB, 32 MiB and 512 MiB and for
    // nearer pairs one chunk per thread stays faster.
    const uint64_t stride_bytes = a.tstride * (C64 ? 8 : 16);
    const bool far = LAYOUT == kSplit &&
                     (stride_bytes == (uint64_t(1) << 28) || stride_bytes >= (uint64_t(1) << 32));
    const int u = a.items > kMaxLaunchItems ? 4 : (far ? 2 : 1);
    const unsigned grid = grid_for(a.items, kBlock * u);
    a.xcd_span = (grid % 8 == 0 && uint64_t(grid) * kBlock * u == a.items) ? grid / 8 : 0;
    if (u == 4)
        hipLaunchKernelGGL((k_pair<C64, LAYOUT, SWAP, NT, 4>), dim3(grid), dim3(kBlock), 0, st, a);
    else if (u == 2)
        hipLaunchKernelGGL((k_pair<C64, LAYOUT, SWAP, NT, 2, true>), dim3(grid), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_pair<C64, LAYOUT, SWAP, NT, 1>), dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <bool C64, int LAYOUT>
hipError_t launch_pair_t(const PairArgs<std::conditional_t<C64, float, double>> &a, bool swap,
                         bool nt, hipStream_t st)
{
    if (a.items == 0) return hipSuccess;
    if (swap)
        return nt ? launch_pair_u<C64, LAYOUT, true, true>(a, st)
                  : launch_pair_u<C64, LAYOUT, true, false>(a, st);
    return nt ? launch_pair_u<C64, LAYOUT, false, true>(a, st)
              : launch_pair_u<C64, LAYOUT, false, false>(a, st);
}

template <bool C64>
hipError_t launch_pair_p(void *psi, int n, int t, uint64_t cmask, const Mat2 &m, bool swap_only,
                         hipStream_t st)
{
    using R = std::conditional_t<C64, float, double>;
    constexpr int lgE = C64 ? 1 : 0;
    constexpr int kLineBit = lgE + 3;                    // amplitude bits inside a 128-byte line
    const uint64_t line_mask = (uint64_t(1) << kLineBit) - 1;
    PairArgs<R> a{};
    a.psi = psi;
    a.tstride = uint64_t(1) << t;
    a.m = to_cmat<R>(m);
    // Controls inside a line are tested per amplitude, so every line the
    // launch touches is read and written whole; controls above it are
    // inserted into the work index as fixed 1 bits, and so is the target
    // (as 0) when the pair spans two lines.
    a.clow = cmask & line_mask;
    // The two halves of a pair sit in lanes of one wave when the target's
    // chunk stride is below 64 (consecutive lanes hold consecutive chunks,
    // and no control inserted into the work index lies below the target):
    // the wave then reads one contiguous run of 1 KiB instead of two streams
    // (30 qubits, complex128 targets 3-5: 6.2 -> 6.7 TB/s).
    constexpr int kWaveBit = lgE + 6;
    const uint64_t below_t = (uint64_t(1) << t) - 1;
    const bool in_wave = t < kWaveBit && !(cmask & ~line_mask & below_t);
    const int layout = t < lgE ? kInChunk : ((t < kLineBit || in_wave) ? kLane : kSplit);
    const uint64_t ins_mask = (layout == kSplit ? a.tstride : 0) | (cmask & ~line_mask);
    int nins = 0;
    for (int b = 0; b < 64; ++b) {
        if (!((ins_mask >> b) & 1)) continue;
        a.pos[nins] = uint8_t(b);
        if (b != t) a.vals |= uint64_t(1) << nins;   // a control: 1; the target: 0
        ++nins;
    }
    a.nins = nins;
    a.items = (uint64_t(1) << n) >> (lgE + nins);
    const bool nt = (uint64_t(1) << n) * (C64 ? 8 : 16) > kStreamBytes;
    if (layout == kSplit) return launch_pair_t<C64, kSplit>(a, swap_only, nt, st);
    if (layout == kLane) return launch_pair_t<C64, kLane>(a, swap_only, nt, st);
    if constexpr (C64) return launch_pair_t<C64, kInChunk>(a, swap_only, nt, st);
    return hipErrorInvalidValue;   // complex128 pairs always span two chunks
}

}  // namespace

hipError_t launch_init(void *psi, int n, sv_dtype dt, uint64_t basis, hipStream_t st)
{
    const uint64_t chunks = (uint64_t(1) << n) >> chunk_log2(dt);
    const unsigned grid = unsigned(std::min<uint64_t>((chunks + kBlock - 1) / kBlock, 8192));
    if (dt == SV_C64) {
        hipLaunchKernelGGL(k_init<true>, dim3(grid), dim3(kBlock), 0, st,
                           InitArgs<true>{psi, chunks, basis});
    } else {
        hipLaunchKernelGGL(k_init<false>, dim3(grid), dim3(kBlock), 0, st,
                           InitArgs<false>{psi, chunks, basis});
    }
    return hipGetLastError();
}

hipError_t launch_pair(void *psi, int n, sv_dtype dt, int t, uint64_t cmask, const Mat2 &m,
                       bool swap_only, hipStream_t st)
{
    return dt == SV_C64 ? launch_pair_p<true>(psi, n, t, cmask, m, swap_only, st)
                        : launch_pair_p<false>(psi, n, t, cmask, m, swap_only, st);
}

hipError_t launch_diag(void *psi, int n, sv_dtype dt, const DiagTerm *terms, int count,
                       hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (count > kMaxDiagTerms) return hipErrorInvalidValue;
    const int lgE = chunk_log2(dt);
    DiagArgs a{};
    a.psi = psi;
    a.count = count;
    uint64_t common = ~uint64_t(0);
    for (int k = 0; k < count; ++k) {
        a.t[k] = terms[k];
        common &= terms[k].mask & terms[k].val;   // bits every term needs set
    }
    // Only bits that select whole 128-byte lines are inserted: lines are read
    // whole, and bits inside a line are left to the per-amplitude terms.
    a.nins = 0;
    for (int b = lgE + 3; b < n && a.nins < 4; ++b)
        if ((common >> b) & 1) a.pos[a.nins++] = b;
    a.items = (uint64_t(1) << n) >> (lgE + a.nins);
    const bool nt = (uint64_t(1) << n) * uint64_t(elem_bytes(dt)) > kStreamBytes;
    auto span = [&](unsigned grid, int u) {
        return (grid % 8 == 0 && uint64_t(grid) * kBlock * u == a.items) ? grid / 8 : 0u;
    };
    if (a.items > kMaxLaunchItems * kDiagU) {     // up to 2^33 chunks: four per thread
        const dim3 grid(grid_for(a.items, kBlock * 4));
        a.xcd_span = span(grid.x, 4);
        if (dt == SV_C64) hipLaunchKernelGGL((k_diag<true, true, 4>), grid, dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_diag<false, true, 4>), grid, dim3(kBlock), 0, st, a);
        return hipGetLastError();
    }
    const dim3 grid(grid_for(a.items, kBlock * kDiagU));
    a.xcd_span = span(grid.x, kDiagU);
    if (dt == SV_C64) {
        if (nt) hipLaunchKernelGGL((k_diag<true, true, kDiagU>), grid, dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_diag<true, false, kDiagU>), grid, dim3(kBlock), 0, st, a);
    } else {
        if (nt) hipLaunchKernelGGL((k_diag<false, true, kDiagU>), grid, dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_diag<false, false, kDiagU>), grid, dim3(kBlock), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace svk
