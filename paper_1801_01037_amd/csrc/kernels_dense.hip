// Dense 5-qubit blocks on the matrix cores.
//
// A run of gates acting only on five qubits B = {b0 < ... < b4} is one 32x32
// complex unitary M (the product of the gates' stride updates restricted to
// those qubits, formed on the host in FP64). Applying it is, for every
// "column" j (a setting of the other n-5 index bits), psi_j <- M psi_j where
// psi_j holds the 32 amplitudes that differ only in the bits of B. With
// X = [Re psi_j ; Im psi_j] (64 rows) and the real 64x64 form
// A = [[Re M, -Im M], [Im M, Re M]], this is Y = A X: a real GEMM of K = 64
// done with 16x16x4 MFMA tiles (FP64 for complex128, FP32 for complex64).
//
// Lane layout of the 16x16x4 MFMAs (lane l of a wave, 0..63): A element
// (row l%16, k l/16), B element (k l/16, column l%16); result register i
// holds column l%16 and row 4*(l/16) + i for the FP32 form but row
// 4*i + l/16 for the FP64 form (read off the hardware with a one-wave probe).
// Each wave takes 16 columns at a time: lane l loads the amplitudes
// r = 4t + l/16 (t = 0..7) of column l%16, runs 4 row tiles x 16 k-steps, and
// stores the amplitudes of the rows its result registers hold.
#include <type_traits>

#include "dense.h"
#include "sv_internal.h"

namespace svk {
namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

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

template <bool C64, bool NT>
__global__ __launch_bounds__(256) void k_dense5(DenseArgs a)
{
    using R = std::conditional_t<C64, float, double>;
    using A2 = std::conditional_t<C64, fv2, dv2>;
    using A4 = std::conditional_t<C64, fv4, dv4>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int l16 = lane & 15, q = lane >> 4;
    const R *mat = static_cast<const R *>(a.mat);   // 64x64 real, row major
    A2 *psi = static_cast<A2 *>(a.psi);

    // This lane's A operands for the 4 row tiles and 16 k-steps.
    R am[4][16];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int s = 0; s < 16; ++s) am[rt][s] = mat[(16 * rt + l16) * 64 + 4 * s + q];

    // Offsets inside a column of the amplitudes this lane loads (r = 4t + q)
    // and stores (the rows of its result registers in row tiles h and h + 2).
    uint64_t in_off[8], out_off[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) in_off[t] = deposit(uint64_t(4 * t + q), a.bmask);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = C64 ? 16 * h + 4 * q + i : 16 * h + 4 * i + q;
            out_off[4 * h + i] = deposit(uint64_t(row), a.bmask);
        }

    const uint64_t ntiles = a.ncols >> 4;
    // Each XCD takes one contiguous eighth of every round of column tiles
    // (scattered 5-qubit blocks at 30 qubits, complex128: 3.8 -> 4.6 TB/s).
    const uint32_t b0 = xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0);
    for (uint64_t tile = uint64_t(b0) * 4 + wave; tile < ntiles; tile += uint64_t(gridDim.x) * 4) {
        const uint64_t base = deposit(tile * 16 + l16, a.omask);
        A2 x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if constexpr (NT) x[t] = __builtin_nontemporal_load(&psi[base | in_off[t]]);
            else x[t] = psi[base | in_off[t]];
        }
        A4 acc[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt] = A4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const R b = s < 8 ? x[s].x : x[s - 8].y;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                if constexpr (C64)
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[rt][s], b, acc[rt], 0, 0, 0);
                else
                    acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[rt][s], b, acc[rt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                A2 y;
                y.x = acc[h][i];
                y.y = acc[h + 2][i];
                if constexpr (NT) __builtin_nontemporal_store(y, &psi[base | out_off[4 * h + i]]);
                else psi[base | out_off[4 * h + i]] = y;
            }
        }
    }
}

// Small registers: work-group g gathers the 2^k amplitudes of its setting of
// the other bits into LDS, thread r forms output r = sum_c U[r][c] x_c in FP64
// and writes it back after every input has been read.
template <bool C64>
__global__ __launch_bounds__(64) void k_unitary_small(SmallUArgs a)
{
    using A2 = std::conditional_t<C64, fv2, dv2>;
    __shared__ dv2 x[32];
    A2 *psi = static_cast<A2 *>(a.psi);
    const dv2 *mat = static_cast<const dv2 *>(a.mat);
    const int r = threadIdx.x;
    for (uint64_t g = blockIdx.x; g < a.ngroups; g += gridDim.x) {
        const uint64_t base = deposit(g, a.omask);
        if (r < a.dim) {
            const A2 v = psi[base | a.off[r]];
            x[r] = dv2{double(v.x), double(v.y)};
        }
        __syncthreads();
        if (r < a.dim) {
            double re = 0.0, im = 0.0;
            for (int c = 0; c < a.dim; ++c) {
                const dv2 u = mat[r * a.dim + c];
                re += u.x * x[c].x - u.y * x[c].y;
                im += u.x * x[c].y + u.y * x[c].x;
            }
            using R = std::conditional_t<C64, float, double>;
            A2 y;
            y.x = R(re);
            y.y = R(im);
            psi[base | a.off[r]] = y;
        }
        __syncthreads();
    }
}

int cus()
{
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
    }
    return n;
}

}  // namespace

hipError_t launch_dense5(const DenseArgs &a, bool c64, hipStream_t st)
{
    const uint64_t tiles = a.ncols >> 4;   // 16 columns per wave step
    if (tiles == 0) return hipErrorInvalidValue;
    const uint64_t want = uint64_t(cus()) * 8;
    const uint64_t blocks_needed = (tiles + 3) / 4;
    const unsigned grid = unsigned(blocks_needed < want ? blocks_needed : want);
    // Streaming hint for states past the last-level cache whose block bits all
    // select whole 128-byte lines (a lane's loads then cover whole lines).
    const int lgE = c64 ? 1 : 0;
    const uint64_t amps = a.ncols << 5;
    const bool nt = amps * (c64 ? 8 : 16) > kStreamBytes && (a.bmask & ((uint64_t(1) << (lgE + 3)) - 1)) == 0;
    if (c64) {
        if (nt) hipLaunchKernelGGL((k_dense5<true, true>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_dense5<true, false>), dim3(grid), dim3(256), 0, st, a);
    } else {
        if (nt) hipLaunchKernelGGL((k_dense5<false, true>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_dense5<false, false>), dim3(grid), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_unitary_small(const SmallUArgs &a, bool c64, hipStream_t st)
{
    if (a.dim < 1 || a.dim > 32 || a.ngroups == 0) return hipErrorInvalidValue;
    const unsigned grid = unsigned(a.ngroups < 4096 ? a.ngroups : 4096);
    if (c64)
        hipLaunchKernelGGL(k_unitary_small<true>, dim3(grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(k_unitary_small<false>, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace svk
