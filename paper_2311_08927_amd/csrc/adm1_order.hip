// Cost order of the persistent step kernel's work queue.
//
// Particles are independent (sec. 4.3, where they are split into equal
// static chunks per thread), but their cost is not: the number of accepted
// and rejected steps per coupling interval spreads over a factor of several
// (fed particles, pH transients).  A queue that hands out particles in index
// order leaves the expensive ones that happen to come last running on
// otherwise idle waves.  The step size h_last proposed at the end of the
// previous interval predicts the cost of the next one, so the queue is
// ordered by the expected step count dt / h_last, largest first, with cold
// particles (no prediction) first of all.  The order is a counting sort over
// kOrderBuckets buckets of width 1/kOrderRes expected steps:
//   k_order_count  -- bucket histogram (LDS per block, one global add per
//                     non-empty bucket and block);
//   k_order_scan   -- one block: descending exclusive prefix sums as the
//                     buckets' first positions; clears the histogram for the
//                     next call and writes the list length for the queue;
//   k_order_place  -- each block ranks its particles per bucket in LDS,
//                     reserves one range per non-empty bucket and scatters.
// The same sort orders an index list whose length is on the device (the
// surrogate's fallback list): element j < *count stands for particle
// list[j].  Ties within a bucket land in an unspecified order; the step
// result of a particle does not depend on where in the queue it is taken.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adm1_kernels.h"

namespace adm1 {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kPerBlock = kThreads * kPerThread;

__device__ __forceinline__ int cost_bucket(double h, double dt)
{
    if (!(h > 0.0)) return kOrderBuckets - 1;
    const double b = dt / h * kOrderRes;
    return b < (double)(kOrderBuckets - 1) ? (int)b : kOrderBuckets - 1;
}

// Length of the list being ordered: n, or *list_count (at most n) with a list.
__device__ __forceinline__ int64_t order_len(int64_t n, const int32_t* list_count)
{
    if (!list_count) return n;
    const int64_t c = list_count[0];
    return c < 0 ? 0 : (c < n ? c : n);
}

__global__ __launch_bounds__(kThreads) void k_order_count(const double* __restrict__ hlast,
                                                          const int32_t* __restrict__ list,
                                                          const int32_t* __restrict__ list_count,
                                                          int64_t n, double dt,
                                                          int32_t* __restrict__ hist)
{
    __shared__ int cnt[kOrderBuckets];
    const int64_t len = order_len(n, list ? list_count : nullptr);
    for (int b = threadIdx.x; b < kOrderBuckets; b += kThreads) cnt[b] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int64_t j = i0 + (int64_t)k * kThreads;
        if (j < len) {
            const int64_t i = list ? (int64_t)list[j] : j;
            atomicAdd(&cnt[cost_bucket(hlast[i], dt)], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderBuckets; b += kThreads) {
        const int c = cnt[b];
        if (c) atomicAdd(&hist[b], c);
    }
}

// One block of kOrderBuckets threads.  Thread t handles bucket
// kOrderBuckets-1-t, so an inclusive scan over t is the descending one.
__global__ __launch_bounds__(kOrderBuckets) void k_order_scan(int32_t* __restrict__ hist,
                                                              int32_t* __restrict__ cursor,
                                                              int32_t* __restrict__ count,
                                                              const int32_t* __restrict__ list_count,
                                                              int64_t n)
{
    __shared__ int buf[2][kOrderBuckets];
    const int t = threadIdx.x;
    const int b = kOrderBuckets - 1 - t;
    const int v = hist[b];
    int cur = 0;
    buf[0][t] = v;
    __syncthreads();
    for (int off = 1; off < kOrderBuckets; off <<= 1) {
        const int x = buf[cur][t] + (t >= off ? buf[cur][t - off] : 0);
        buf[cur ^ 1][t] = x;
        cur ^= 1;
        __syncthreads();
    }
    cursor[b] = buf[cur][t] - v;
    hist[b] = 0;
    if (t == 0) count[0] = (int32_t)order_len(n, list_count);
}

__global__ __launch_bounds__(kThreads) void k_order_place(const double* __restrict__ hlast,
                                                          const int32_t* __restrict__ list,
                                                          const int32_t* __restrict__ list_count,
                                                          int64_t n, double dt,
                                                          int32_t* __restrict__ cursor,
                                                          int32_t* __restrict__ order)
{
    __shared__ int cnt[kOrderBuckets];
    __shared__ int base[kOrderBuckets];
    const int64_t len = order_len(n, list ? list_count : nullptr);
    for (int b = threadIdx.x; b < kOrderBuckets; b += kThreads) cnt[b] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPerBlock + threadIdx.x;
    int bk[kPerThread], rk[kPerThread], id[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int64_t j = i0 + (int64_t)k * kThreads;
        bk[k] = 0;
        rk[k] = 0;
        id[k] = -1;
        if (j < len) {
            id[k] = list ? list[j] : (int32_t)j;
            bk[k] = cost_bucket(hlast[id[k]], dt);
            rk[k] = atomicAdd(&cnt[bk[k]], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kOrderBuckets; b += kThreads) {
        const int c = cnt[b];
        base[b] = c ? atomicAdd(&cursor[b], c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPerThread; ++k)
        if (id[k] >= 0) order[base[bk[k]] + rk[k]] = id[k];
}

}  // namespace

hipError_t launch_cost_order(const double* hlast, const int32_t* list,
                             const int32_t* list_count, int64_t n, double dt, int32_t* work,
                             int32_t* order, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (!list) list_count = nullptr;
    int32_t* hist = work;
    int32_t* cursor = work + kOrderBuckets;
    int32_t* count = work + 2 * kOrderBuckets;
    const unsigned grid = (unsigned)((n + kPerBlock - 1) / kPerBlock);
    hipLaunchKernelGGL(k_order_count, dim3(grid), dim3(kThreads), 0, s, hlast, list, list_count,
                       n, dt, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBuckets), 0, s, hist, cursor, count,
                       list_count, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_place, dim3(grid), dim3(kThreads), 0, s, hlast, list, list_count,
                       n, dt, cursor, order);
    return hipGetLastError();
}

}  // namespace adm1
