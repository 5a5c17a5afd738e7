// Per-gate kernels: basis-state init, the 2x2 pair update (plain, controlled,
// exchange-only) and diagonal runs.
//
// The pair update is the stride rule of State Vector Partitioning: for a gate
// on qubit t every pair (i0, i0 + 2^t) with bit t of i0 clear becomes
// (q11 a + q12 b, q21 a + q22 b); a control c restricts it to indices with bit
// c set (caption of Algorithm 1), several controls (a Toffoli gate has two) to
// indices with all of them set. Instead of the paper's two nested loops, a
// flat work index is expanded by inserting the fixed bits (target = 0,
// controls = 1), so consecutive lanes touch consecutive 16-byte chunks of both
// halves of every pair and both streams are coalesced for any t.
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

// Where the two amplitudes of a pair sit relative to 16-byte chunks.
enum Layout {
    kSplit = 0,     // a and b in different chunks, 2^t apart; every amp of a chunk pairs
    kInChunk = 1,   // c64, t = 0: one chunk holds (a, b)
    kSplitOdd = 2,  // c64, control 0: split chunks, only the odd amplitude is controlled on
};

template <typename R>
struct PairArgs {
    void *psi;
    uint64_t items;       // work items (chunk pairs, or chunks for kInChunk)
    uint64_t tstride;     // 2^t in amplitudes
    int nins;             // fixed index bits to insert, ascending positions
    uint64_t vals;        // bit k: the value inserted at pos[k]
    CMat<R> m;
    uint8_t pos[64];
};

template <bool C64, int LAYOUT, bool SWAP, int U>
__global__ __launch_bounds__(kBlock) void k_pair(PairArgs<std::conditional_t<C64, float, double>> a)
{
    using R = std::conditional_t<C64, float, double>;
    using V = std::conditional_t<C64, float4, double2>;   // one 16-byte chunk
    constexpr uint64_t E = C64 ? 2 : 1;                   // amplitudes per chunk
    V *p = static_cast<V *>(a.psi);
    const uint64_t first = uint64_t(blockIdx.x) * (kBlock * U) + threadIdx.x;

    V va[U], vb[U];
    uint64_t ca[U], cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        uint64_t x = item * E;
        for (int k = 0; k < a.nins; ++k) x = insert_bit(x, a.pos[k], (a.vals >> k) & 1u);
        ca[u] = x / E;
        cb[u] = (x + a.tstride) / E;
        if (item < a.items) {
            va[u] = p[ca[u]];
            if (LAYOUT != kInChunk) vb[u] = p[cb[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        if (item >= a.items) continue;
        if constexpr (C64) {
            if constexpr (LAYOUT == kSplit) {
                if constexpr (SWAP) {
                    V t = va[u]; va[u] = vb[u]; vb[u] = t;
                } else {
                    pair_update<R>(va[u].x, va[u].y, vb[u].x, vb[u].y, a.m);
                    pair_update<R>(va[u].z, va[u].w, vb[u].z, vb[u].w, a.m);
                }
            } else if constexpr (LAYOUT == kInChunk) {
                if constexpr (SWAP) {
                    va[u] = make_float4(va[u].z, va[u].w, va[u].x, va[u].y);
                } else {
                    pair_update<R>(va[u].x, va[u].y, va[u].z, va[u].w, a.m);
                }
            } else {  // kSplitOdd
                if constexpr (SWAP) {
                    R z = va[u].z, w = va[u].w;
                    va[u].z = vb[u].z; va[u].w = vb[u].w;
                    vb[u].z = z; vb[u].w = w;
                } else {
                    pair_update<R>(va[u].z, va[u].w, vb[u].z, vb[u].w, a.m);
                }
            }
        } else {
            if constexpr (SWAP) {
                V t = va[u]; va[u] = vb[u]; vb[u] = t;
            } else {
                pair_update<R>(va[u].x, va[u].y, vb[u].x, vb[u].y, a.m);
            }
        }
        p[ca[u]] = va[u];
        if (LAYOUT != kInChunk) p[cb[u]] = vb[u];
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
    for (uint64_t c = uint64_t(blockIdx.x) * kBlock + threadIdx.x; c < a.chunks; c += stride) {
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
    int nins;             // bits fixed to 1 in every visited index (ascending)
    int pos[4];
    int count;
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

template <bool C64, int U>
__global__ __launch_bounds__(kBlock) void k_diag(DiagArgs a)
{
    using V = std::conditional_t<C64, float4, double2>;
    constexpr uint64_t E = C64 ? 2 : 1;
    V *p = static_cast<V *>(a.psi);
    const uint64_t first = uint64_t(blockIdx.x) * (kBlock * U) + threadIdx.x;
    V v[U];
    uint64_t ci[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        uint64_t x = item * E;
        for (int k = 0; k < a.nins; ++k) x = insert_bit(x, a.pos[k], 1);
        ci[u] = x / E;
        if (item < a.items) v[u] = p[ci[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t item = first + uint64_t(u) * kBlock;
        if (item >= a.items) continue;
        const uint64_t i0 = ci[u] * E;
        if constexpr (C64) {
            const uint64_t T0 = turn_of(i0, a), T1 = turn_of(i0 + 1, a);
            if ((T0 | T1) == 0) continue;
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
            if (T == 0) continue;
            double c, s;
            turn_phase(T, c, s);
            const double re = v[u].x * c - v[u].y * s;
            const double im = v[u].x * s + v[u].y * c;
            v[u].x = re; v[u].y = im;
        }
        p[ci[u]] = v[u];
    }
}

constexpr int kPairU = 4;
constexpr int kDiagU = 2;

inline unsigned grid_for(uint64_t items, int per_block)
{
    return unsigned((items + per_block - 1) / per_block);
}

template <bool C64, int LAYOUT, bool SWAP>
hipError_t launch_pair_t(const PairArgs<std::conditional_t<C64, float, double>> &a,
                         hipStream_t st)
{
    if (a.items == 0) return hipSuccess;
    hipLaunchKernelGGL((k_pair<C64, LAYOUT, SWAP, kPairU>), dim3(grid_for(a.items, kBlock * kPairU)),
                       dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <bool C64>
hipError_t launch_pair_p(void *psi, int n, int t, uint64_t cmask, const Mat2 &m, bool swap_only,
                         hipStream_t st)
{
    using R = std::conditional_t<C64, float, double>;
    constexpr int lgE = C64 ? 1 : 0;
    PairArgs<R> a{};
    a.psi = psi;
    a.tstride = uint64_t(1) << t;
    a.m = to_cmat<R>(m);
    // Fixed bits inserted into the work index, ascending: the target bit (0)
    // when the pair spans two chunks, every control bit (1) that is constant
    // over a chunk. A complex64 control on bit 0 selects the odd amplitude of
    // each chunk instead (kSplitOdd).
    int layout;
    if (t >= lgE) {
        layout = (lgE > 0 && (cmask & 1u)) ? kSplitOdd : kSplit;
    } else {
        layout = kInChunk;
    }
    const uint64_t ins_mask = (layout != kInChunk ? (uint64_t(1) << t) : 0) |
                              (cmask & ~((uint64_t(1) << lgE) - 1));
    int nins = 0;
    for (int b = 0; b < 64; ++b) {
        if (!((ins_mask >> b) & 1)) continue;
        a.pos[nins] = uint8_t(b);
        if (b != t) a.vals |= uint64_t(1) << nins;   // a control: 1; the target: 0
        ++nins;
    }
    a.nins = nins;
    a.items = (uint64_t(1) << n) >> (lgE + nins);
    if (layout == kSplit)
        return swap_only ? launch_pair_t<C64, kSplit, true>(a, st)
                         : launch_pair_t<C64, kSplit, false>(a, st);
    if (layout == kInChunk)
        return swap_only ? launch_pair_t<C64, kInChunk, true>(a, st)
                         : launch_pair_t<C64, kInChunk, false>(a, st);
    return swap_only ? launch_pair_t<C64, kSplitOdd, true>(a, st)
                     : launch_pair_t<C64, kSplitOdd, false>(a, st);
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
    a.nins = 0;
    for (int b = lgE; b < n && a.nins < 4; ++b)
        if ((common >> b) & 1) a.pos[a.nins++] = b;
    a.items = (uint64_t(1) << n) >> (lgE + a.nins);
    const unsigned grid = grid_for(a.items, kBlock * kDiagU);
    if (dt == SV_C64)
        hipLaunchKernelGGL((k_diag<true, kDiagU>), dim3(grid), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_diag<false, kDiagU>), dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace svk
