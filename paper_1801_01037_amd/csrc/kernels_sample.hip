// Measurement sampling and the uniform initial state.
//
// Sampling draws basis indices with probability |alpha_i|^2 / norm (the
// measurement symbols of section Quantum Circuits): for each caller-supplied
// uniform u in [0, 1), sorted ascending, the index i with
//     CDF(i - 1) <= u * norm < CDF(i),   CDF(i) = sum_{k <= i} |alpha_k|^2.
// The state is cut into blocks of 2^12 amplitudes. One pass forms every
// block's FP64 sum, one small launch their exclusive prefix (P[nb] = norm),
// and one work-group per block that received samples scans the block's
// probabilities in LDS and binary-searches each of its samples there. The
// state is read once for the sums and once more for the blocks that hold
// samples.
//
// The uniform state 2^{-n/2} sum_x |x> (H on every qubit of |0...0>, section
// Quantum Information Processing) is one write of the state.
#include <mutex>
#include <type_traits>

#include "sv_internal.h"

// Sampling scratch for callers that cannot allocate device memory: block sums
// and their prefix for states of up to kStaticSampleMaxQubits qubits (4 MiB).
// Each GPU holds its own copy until the process ends. In host code this name
// stands for a host-side shadow, not a device address: host code passes the
// address that static_sample_scratch looks up, never the name itself.
static __device__ __align__(256) double scratch[svk::sample_scratch_doubles(svk::kStaticSampleMaxQubits)];

namespace svk {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = kSampleBlock / kThreads;   // 16

template <bool C64>
__device__ __forceinline__ double prob_at(const void *psi, uint64_t i)
{
    if constexpr (C64) {
        const float2 a = static_cast<const float2 *>(psi)[i];
        return double(a.x) * double(a.x) + double(a.y) * double(a.y);
    } else {
        const double2 a = static_cast<const double2 *>(psi)[i];
        return a.x * a.x + a.y * a.y;
    }
}

// S[b] = sum of |alpha|^2 over block b (bsize amplitudes); a fixed tree, so
// the same state gives the same bits every time.
template <bool C64>
__global__ __launch_bounds__(kThreads) void k_block_sums(const void *psi, uint64_t nb, int bsize,
                                                          double *S)
{
    using V = std::conditional_t<C64, float4, double2>;   // one 16-byte chunk
    constexpr int E = C64 ? 2 : 1;
    const V *p = static_cast<const V *>(psi);
    __shared__ double part[kThreads];
    // Each XCD takes one contiguous eighth of every round of blocks.
    const uint64_t b0 = xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0);
    for (uint64_t b = b0; b < nb; b += gridDim.x) {
        const uint64_t base = b * uint64_t(bsize / E);
        double s = 0.0;
        for (int k = threadIdx.x; k < bsize / E; k += kThreads) {
            const V v = p[base + k];
            if constexpr (C64) {
                const double a = v.x, c = v.y, d = v.z, e = v.w;
                s += (a * a + c * c) + (d * d + e * e);
            } else {
                s += v.x * v.x + v.y * v.y;
            }
        }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) S[b] = part[0];
        __syncthreads();
    }
}

// P[b] = sum_{b' < b} S[b'] for b <= nb (P[nb] is the norm), and P[nb + 1]
// = the last block with a non-zero sum (as a double; 0 if none). One
// work-group of 1024 threads: each sums a contiguous run of S, the run totals
// are scanned in LDS, and each thread writes its run's prefixes.
__global__ __launch_bounds__(1024) void k_scan_blocks(const double *S, uint64_t nb, double *P)
{
    __shared__ double tot[1024];
    __shared__ int64_t lastnz[1024];
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t lo = uint64_t(threadIdx.x) * per;
    const uint64_t hi = lo + per < nb ? lo + per : nb;
    double s = 0.0;
    int64_t lz = -1;
    for (uint64_t b = lo; b < hi; ++b) {
        s += S[b];
        if (S[b] > 0.0) lz = int64_t(b);
    }
    tot[threadIdx.x] = s;
    lastnz[threadIdx.x] = lz;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        int64_t last = 0;
        for (int t = 0; t < 1024; ++t) {
            const double v = tot[t];
            tot[t] = run;
            run += v;
            if (lastnz[t] >= 0) last = lastnz[t];
        }
        P[nb] = run;
        P[nb + 1] = double(last);
    }
    __syncthreads();
    double run = tot[threadIdx.x];
    for (uint64_t b = lo; b < hi; ++b) {
        P[b] = run;
        run += S[b];
    }
}

// First j in [0, m) with u[j] * norm >= x (m if none); u ascending.
__device__ __forceinline__ uint64_t first_at_least(const double *u, uint64_t m, double norm, double x)
{
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (u[mid] * norm < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <bool C64>
__global__ __launch_bounds__(kThreads) void k_sample(const void *psi, uint64_t nb, int bsize,
                                                      const double *P, const double *u, uint64_t m,
                                                      uint64_t *out)
{
    __shared__ double pre[kSampleBlock];   // inclusive prefix of the block's probabilities
    __shared__ double tsum[kThreads];
    __shared__ uint64_t range[2];
    const double norm = P[nb];
    const uint64_t lastnz = uint64_t(P[nb + 1]);
    for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        if (threadIdx.x == 0) {
            // The last block with a non-zero sum also takes the samples that
            // rounding put at or above the norm; blocks after it take none.
            range[0] = b > lastnz ? m : first_at_least(u, m, norm, P[b]);
            range[1] = b >= lastnz ? m : first_at_least(u, m, norm, P[b + 1]);
        }
        __syncthreads();
        const uint64_t lo = range[0], hi = range[1];
        if (lo < hi) {
            // Each thread scans kPerThread consecutive probabilities; thread
            // totals are scanned by thread 0; then offsets are added.
            const uint64_t base = b * uint64_t(bsize);
            const int k0 = int(threadIdx.x) * kPerThread;
            double run = 0.0;
            for (int k = 0; k < kPerThread; ++k) {
                const double p = k0 + k < bsize ? prob_at<C64>(psi, base + k0 + k) : 0.0;
                run += p;
                pre[k0 + k] = run;
            }
            tsum[threadIdx.x] = run;
            __syncthreads();
            if (threadIdx.x == 0) {
                double acc = 0.0;
                for (int t = 0; t < kThreads; ++t) {
                    const double v = tsum[t];
                    tsum[t] = acc;
                    acc += v;
                }
            }
            __syncthreads();
            const double off = tsum[threadIdx.x];
            for (int k = 0; k < kPerThread; ++k) pre[k0 + k] += off;
            __syncthreads();
            for (uint64_t j = lo + threadIdx.x; j < hi; j += kThreads) {
                const double target = u[j] * norm - P[b];
                // first k with pre[k] > target: its probability is positive
                int a = 0, c = bsize;
                while (a < c) {
                    const int mid = (a + c) >> 1;
                    if (pre[mid] <= target) a = mid + 1;
                    else c = mid;
                }
                if (a == bsize) {   // rounding past the block's scanned total:
                    a = bsize - 1;  // its last amplitude of non-zero probability
                    while (a > 0 && pre[a] == pre[a - 1]) --a;
                }
                out[j] = base + uint64_t(a);
            }
        }
        __syncthreads();
    }
}

template <bool C64>
__global__ __launch_bounds__(kThreads) void k_fill(void *psi, uint64_t count, double value)
{
    // count: 16-byte chunks (two complex64 or one complex128 amplitude each);
    // each XCD writes one contiguous eighth of every grid stride.
    using V = std::conditional_t<C64, float4, double2>;
    V v;
    if constexpr (C64) v = make_float4(float(value), 0.f, float(value), 0.f);
    else v = make_double2(value, 0.0);
    V *p = static_cast<V *>(psi);
    const uint64_t b = xcd_block(blockIdx.x, gridDim.x % 8 == 0 ? gridDim.x / 8 : 0);
    for (uint64_t i = b * kThreads + threadIdx.x; i < count; i += uint64_t(gridDim.x) * kThreads)
        p[i] = v;
}

unsigned grid_of(uint64_t items, uint64_t cap)
{
    return unsigned(items < cap ? (items ? items : 1) : cap);
}

}  // namespace

hipError_t static_sample_scratch(int device, double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_block_sums(const void *psi, int n, sv_dtype dt, double *S, hipStream_t st)
{
    const int bsize = n < kSampleBlockLog ? (1 << n) : kSampleBlock;
    const uint64_t nb = (uint64_t(1) << n) / uint64_t(bsize);
    const unsigned grid = grid_of(nb, 65536);
    if (dt == SV_C64) hipLaunchKernelGGL(k_block_sums<true>, dim3(grid), dim3(kThreads), 0, st, psi, nb, bsize, S);
    else hipLaunchKernelGGL(k_block_sums<false>, dim3(grid), dim3(kThreads), 0, st, psi, nb, bsize, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, S, nb, S + nb);
    return hipGetLastError();
}

hipError_t launch_sample(const void *psi, int n, sv_dtype dt, const double *S, const double *u,
                         uint64_t m, uint64_t *out, hipStream_t st)
{
    const int bsize = n < kSampleBlockLog ? (1 << n) : kSampleBlock;
    const uint64_t nb = (uint64_t(1) << n) / uint64_t(bsize);
    const double *P = S + nb;
    const unsigned grid = grid_of(nb, 65536);
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_sample<true>, dim3(grid), dim3(kThreads), 0, st, psi, nb, bsize, P, u, m, out);
    else
        hipLaunchKernelGGL(k_sample<false>, dim3(grid), dim3(kThreads), 0, st, psi, nb, bsize, P, u, m, out);
    return hipGetLastError();
}

hipError_t launch_fill(void *psi, int n, sv_dtype dt, double value, hipStream_t st)
{
    const uint64_t count = (uint64_t(1) << n) >> chunk_log2(dt);   // n >= 1: whole chunks
    const unsigned grid = grid_of((count + kThreads - 1) / kThreads, 8192);
    if (dt == SV_C64) hipLaunchKernelGGL(k_fill<true>, dim3(grid), dim3(kThreads), 0, st, psi, count, value);
    else hipLaunchKernelGGL(k_fill<false>, dim3(grid), dim3(kThreads), 0, st, psi, count, value);
    return hipGetLastError();
}

}  // namespace svk
