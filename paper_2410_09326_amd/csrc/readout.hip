// Two-qubit Z correlators <Z_a Z_b> = sum_x |psi_x|^2 (-1)^(x_a + x_b) for
// lists of physical bit pairs: the expectation values a diagonal cost
// Hamiltonian (weighted Max-Cut in repeated QAOA runs, paper Sec. IV-E) is
// assembled from.  One sweep over the state per chunk of eight pairs, FP64
// accumulation with a fixed summation order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace qops {
namespace {

constexpr int kZZChunk = 8;
constexpr int kZZThreads = 256;

struct PairChunk {
    int32_t a[kZZChunk];
    int32_t b[kZZChunk];
    int32_t count;
};

template <typename T>
struct Amp;
template <>
struct Amp<float> {
    using V = float2;
};
template <>
struct Amp<double> {
    using V = double2;
};

// Tree sum of the 256 values in sh (every thread has written its own); the
// result is in sh[0] after the last barrier.
__device__ __forceinline__ void tree_sum_256(double* sh)
{
    for (int s = kZZThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
}

// Block g sums amplitudes [g * per, (g + 1) * per) (threads stride by 256)
// and writes one partial per pair of the chunk: part[g * 8 + c].
template <typename T>
__global__ void __launch_bounds__(kZZThreads)
zz_part_kernel(const typename Amp<T>::V* __restrict__ st, uint64_t N, uint64_t per, PairChunk pc,
               double* __restrict__ part)
{
    __shared__ double sh[kZZThreads];
    double acc[kZZChunk];
#pragma unroll
    for (int c = 0; c < kZZChunk; ++c) acc[c] = 0.0;
    const uint64_t x0 = (uint64_t)blockIdx.x * per;
    const uint64_t x1 = x0 + per < N ? x0 + per : N;
    for (uint64_t x = x0 + threadIdx.x; x < x1; x += kZZThreads) {
        const typename Amp<T>::V v = st[x];
        const double p = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
#pragma unroll
        for (int c = 0; c < kZZChunk; ++c) {
            if (c < pc.count) {
                const uint64_t s = ((x >> pc.a[c]) ^ (x >> pc.b[c])) & 1ull;
                acc[c] += s ? -p : p;
            }
        }
    }
    for (int c = 0; c < pc.count; ++c) {
        sh[threadIdx.x] = acc[c];
        __syncthreads();
        tree_sum_256(sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kZZChunk + c] = sh[0];
        __syncthreads();
    }
}

// out[c] = sum over blocks g of part[g * 8 + c], in a fixed order.
__global__ void __launch_bounds__(kZZThreads)
zz_final_kernel(const double* __restrict__ part, int nblocks, double* __restrict__ out)
{
    __shared__ double sh[kZZThreads];
    const int c = blockIdx.x;
    double v = 0.0;
    for (int g = threadIdx.x; g < nblocks; g += kZZThreads) v += part[(size_t)g * kZZChunk + c];
    sh[threadIdx.x] = v;
    __syncthreads();
    tree_sum_256(sh);
    if (threadIdx.x == 0) out[c] = sh[0];
}

}  // namespace

size_t zz_scratch_doubles(int n)
{
    const uint64_t N = 1ull << n;
    const uint64_t nb = std::max<uint64_t>(1, std::min<uint64_t>(4096, N / kZZThreads));
    return (size_t)nb * kZZChunk;
}

hipError_t launch_expect_zz(int prec, const void* state, int n, const int32_t* pa, const int32_t* pb, int npairs,
                            double* part, double* d_out, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const uint64_t nb = std::max<uint64_t>(1, std::min<uint64_t>(4096, N / kZZThreads));
    const uint64_t per = (N + nb - 1) / nb;
    for (int p0 = 0; p0 < npairs; p0 += kZZChunk) {
        PairChunk pc;
        pc.count = std::min(kZZChunk, npairs - p0);
        for (int c = 0; c < kZZChunk; ++c) {
            pc.a[c] = c < pc.count ? pa[p0 + c] : 0;
            pc.b[c] = c < pc.count ? pb[p0 + c] : 0;
        }
        if (prec == 0)
            hipLaunchKernelGGL(zz_part_kernel<float>, dim3((unsigned)nb), dim3(kZZThreads), 0, s,
                               reinterpret_cast<const float2*>(state), N, per, pc, part);
        else
            hipLaunchKernelGGL(zz_part_kernel<double>, dim3((unsigned)nb), dim3(kZZThreads), 0, s,
                               reinterpret_cast<const double2*>(state), N, per, pc, part);
        hipLaunchKernelGGL(zz_final_kernel, dim3((unsigned)pc.count), dim3(kZZThreads), 0, s, part, (int)nb,
                           d_out + p0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qops
