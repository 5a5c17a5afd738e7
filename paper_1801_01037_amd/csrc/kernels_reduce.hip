// Norm and probability reductions. Squares and sums are formed in FP64 for
// both storage precisions (the normalisation condition sum |alpha_i|^2 = 1 of
// Quantum Information Processing).
//
// The norm is a fixed two-level tree: kNormBlocks blocks each sum a fixed,
// strided subset of the 16-byte chunks (thread-sequential, then a wave
// shuffle tree, then across waves), and one block sums the partials in a
// fixed order. No floating-point atomics, so a state gives the same bits on
// every call.
#include <type_traits>

#include "sv_internal.h"

namespace svk {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of `kThreads` threads; result valid in thread 0.
template <int kThreads>
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[kThreads / 64];
    v = wave_sum(v);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) s += part[w];
    return s;
}

template <bool C64, bool NT>
__global__ __launch_bounds__(kBlock) void k_norm_partial(const void *psi, uint64_t chunks,
                                                         double *partials)
{
    using V = std::conditional_t<C64, float4, double2>;
    const V *p = static_cast<const V *>(psi);
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    auto sq = [](const V &v) -> double {
        if constexpr (C64) {
            const double a = v.x, b = v.y, d = v.z, e = v.w;
            return (a * a + b * b) + (d * d + e * e);
        } else {
            return v.x * v.x + v.y * v.y;
        }
    };
    // Four loads in flight per thread, four partial sums; each XCD walks one
    // contiguous eighth of every stride (complex64: 5.4 -> 6.3 TB/s).
    double acc = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    uint64_t c = uint64_t(xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0)) * kBlock +
                 threadIdx.x;
    for (; c + 3 * stride < chunks; c += 4 * stride) {
        const V v0 = ld16<NT>(&p[c]), v1 = ld16<NT>(&p[c + stride]);
        const V v2 = ld16<NT>(&p[c + 2 * stride]), v3 = ld16<NT>(&p[c + 3 * stride]);
        acc += sq(v0);
        acc1 += sq(v1);
        acc2 += sq(v2);
        acc3 += sq(v3);
    }
    for (; c < chunks; c += stride) acc += sq(ld16<NT>(&p[c]));
    acc = (acc + acc1) + (acc2 + acc3);
    const double s = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kNormBlocks) void k_norm_final(const double *partials, double *out)
{
    const double s = block_sum<kNormBlocks>(partials[threadIdx.x]);
    if (threadIdx.x == 0) *out = s;
}

// Two amplitudes (2p, 2p + 1) of a state, widened to FP64.
template <bool C64, bool NT>
__device__ __forceinline__ void load_pair(const void *psi, uint64_t p, double (&v)[4])
{
    if constexpr (C64) {
        const float4 a = ld16<NT>(static_cast<const float4 *>(psi) + p);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
        const double2 *q = static_cast<const double2 *>(psi) + 2 * p;
        const double2 a = ld16<NT>(q), b = ld16<NT>(q + 1);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// The four comparison figures of one thread, reduced over the block: thread
// k < 4 writes figure k to out[k * stride]. Figures: 0 the largest
// |a_i - b_i|^2, 1 sum |a_i - b_i|^2, 2 sum |a_i|^2, 3 sum |b_i|^2.
template <int kThreads>
__device__ __forceinline__ void block_compare(double (&r)[4], double *out, uint32_t stride)
{
    __shared__ double w[4][kThreads / 64];
    r[0] = wave_max(r[0]);
    for (int k = 1; k < 4; ++k) r[k] = wave_sum(r[k]);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
        for (int k = 0; k < 4; ++k) w[k][wave] = r[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double s = w[k][0];
        for (int i = 1; i < kThreads / 64; ++i) s = k == 0 ? fmax(s, w[k][i]) : s + w[k][i];
        out[k * stride] = s;
    }
}

// The error of state a against state b (same length, either precision), all
// in FP64: a fixed-shape reduction like the norm's (the same bits every call).
// Block b's figures go to part[k * kNormBlocks + b].
template <bool AC64, bool BC64, bool NT>
__global__ __launch_bounds__(kBlock) void k_compare_partial(const void *a, const void *b,
                                                            uint64_t pairs, double *part)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    uint64_t p = uint64_t(xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0)) * kBlock +
                 threadIdx.x;
    for (; p < pairs; p += stride) {
        double x[4], y[4];
        load_pair<AC64, NT>(a, p, x);
        load_pair<BC64, NT>(b, p, y);
        for (int h = 0; h < 4; h += 2) {
            const double dr = x[h] - y[h], di = x[h + 1] - y[h + 1];
            const double d2 = dr * dr + di * di;
            r[0] = fmax(r[0], d2);
            r[1] += d2;
            r[2] += x[h] * x[h] + x[h + 1] * x[h + 1];
            r[3] += y[h] * y[h] + y[h + 1] * y[h + 1];
        }
    }
    block_compare<kBlock>(r, part + blockIdx.x, kNormBlocks);
}

// out[0] = max |a_i - b_i|, out[1..3] the three sums.
__global__ __launch_bounds__(kNormBlocks) void k_compare_final(const double *part, double *out)
{
    double r[4];
    for (int k = 0; k < 4; ++k) r[k] = part[k * kNormBlocks + threadIdx.x];
    block_compare<kNormBlocks>(r, out, 1);
    if (threadIdx.x == 0) out[0] = sqrt(out[0]);   // thread 0 wrote out[0] itself
}

template <bool C64>
__global__ __launch_bounds__(kBlock) void k_probs(const void *psi, uint64_t first,
                                                  uint64_t count, double *out)
{
    using A = std::conditional_t<C64, float2, double2>;
    const A *p = static_cast<const A *>(psi) + first;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        const A v = p[i];
        const double re = v.x, im = v.y;
        out[i] = re * re + im * im;
    }
}

}  // namespace

hipError_t launch_norm(const void *psi, int n, sv_dtype dt, double *partials, double *out_dev,
                       hipStream_t st)
{
    const uint64_t chunks = (uint64_t(1) << n) >> chunk_log2(dt);
    const bool nt = (uint64_t(1) << n) * uint64_t(elem_bytes(dt)) > kStreamBytes;
    const dim3 grid(kNormBlocks), block(kBlock);
    if (dt == SV_C64) {
        if (nt) hipLaunchKernelGGL((k_norm_partial<true, true>), grid, block, 0, st, psi, chunks, partials);
        else hipLaunchKernelGGL((k_norm_partial<true, false>), grid, block, 0, st, psi, chunks, partials);
    } else {
        if (nt) hipLaunchKernelGGL((k_norm_partial<false, true>), grid, block, 0, st, psi, chunks, partials);
        else hipLaunchKernelGGL((k_norm_partial<false, false>), grid, block, 0, st, psi, chunks, partials);
    }
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kNormBlocks), 0, st, partials, out_dev);
    return hipGetLastError();
}

hipError_t launch_compare(const void *a, sv_dtype da, const void *b, sv_dtype db, int n,
                          double *scratch, hipStream_t st)
{
    const uint64_t pairs = uint64_t(1) << (n - 1);
    const uint64_t bytes = (uint64_t(1) << n) * uint64_t(elem_bytes(da) + elem_bytes(db));
    const bool nt = bytes > kStreamBytes;
    const dim3 grid(kNormBlocks), block(kBlock);
#define SV_CMP(A, B)                                                                            \
    do {                                                                                      \
        if (nt) hipLaunchKernelGGL((k_compare_partial<A, B, true>), grid, block, 0, st, a, b,  \
                                   pairs, scratch);                                           \
        else hipLaunchKernelGGL((k_compare_partial<A, B, false>), grid, block, 0, st, a, b,    \
                                pairs, scratch);                                              \
    } while (0)
    if (da == SV_C64) {
        if (db == SV_C64) SV_CMP(true, true);
        else SV_CMP(true, false);
    } else {
        if (db == SV_C64) SV_CMP(false, true);
        else SV_CMP(false, false);
    }
#undef SV_CMP
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compare_final, dim3(1), dim3(kNormBlocks), 0, st, scratch,
                       scratch + 4 * kNormBlocks);
    return hipGetLastError();
}

hipError_t launch_probs(const void *psi, sv_dtype dt, uint64_t first, uint64_t count,
                        double *out_dev, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    const unsigned grid = unsigned(std::min<uint64_t>((count + kBlock - 1) / kBlock, 16384));
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_probs<true>, dim3(grid), dim3(kBlock), 0, st, psi, first, count,
                           out_dev);
    else
        hipLaunchKernelGGL(k_probs<false>, dim3(grid), dim3(kBlock), 0, st, psi, first, count,
                           out_dev);
    return hipGetLastError();
}

}  // namespace svk
