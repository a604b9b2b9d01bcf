// Data handling of the surrogate's training driver on the device: row
// gathers for mini-batches, a seeded permutation of the rows per epoch, and
// FP64 column statistics (input / target normalisation, the mean residual
// and the mean squared error of the network).  Reductions run in a fixed
// order (per-block partials, then one ordered pass), so every statistic is
// reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "adm1.h"
#include "adm1_ctx.h"

using namespace adm1_abi;

namespace {

constexpr int kStatBlocks = 1024;   // partial sums per statistic pass
constexpr int kStatThreads = 256;   // 4 row lanes of 64 columns
constexpr int kMaxCols = 64;

// ---------------------------------------------------------------------------
// Row gather: dst row j = src row idx[j], rows of `words` 4-byte words; an
// index outside [0, n_src) yields a zero row.
// ---------------------------------------------------------------------------
__global__ void k_gather(const uint32_t* __restrict__ src, int64_t n_src, int64_t words,
                         const int32_t* __restrict__ idx, int64_t n_idx, uint32_t* __restrict__ dst)
{
    const int64_t total = n_idx * words;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = w / words, k = w - j * words;
        const int64_t r = idx[j];
        dst[w] = (r >= 0 && r < n_src) ? src[r * words + k] : 0u;
    }
}

// ---------------------------------------------------------------------------
// Seeded permutation of [0, n): a four-round balanced Feistel network on
// 2 h bits (the smallest even width with 2^(2h) >= n) is a bijection of
// [0, 2^(2h)); cycle walking (re-encrypting until the value falls below n)
// restricts it to a bijection of [0, n).  The walk from i < n stays on i's
// cycle, which returns below n, so it ends.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

struct Feistel {
    uint32_t keys[4];
    int half;       // bits per half
    uint32_t mask;  // (1 << half) - 1
    __device__ uint64_t enc(uint64_t x) const
    {
        uint32_t l = (uint32_t)(x >> half) & mask, r = (uint32_t)x & mask;
        for (int k = 0; k < 4; ++k) {
            const uint32_t t = l ^ (mix32(r ^ keys[k]) & mask);
            l = r;
            r = t;
        }
        return ((uint64_t)l << half) | r;
    }
};

__global__ void k_permutation(Feistel f, int64_t n, int32_t* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t y = f.enc((uint64_t)i);
        while (y >= (uint64_t)n) y = f.enc(y);
        out[i] = (int32_t)y;
    }
}

// ---------------------------------------------------------------------------
// Column sums.  Thread t of a block takes column t % 64 of every fourth row
// of the block's rows (rows b, b + B, ...); the block's four row lanes are
// added in a fixed order; partial[block][col] holds the block's sum.  Value
// of (row, col): a float32 or BF16 element, minus center[col] and squared
// when `square` is set.
// ---------------------------------------------------------------------------
struct ColSrc {
    const void* data;
    int32_t bf16;    // 1: BF16 bit patterns, 0: float32
    int64_t ld;      // elements per row
};

__device__ inline double col_value(const ColSrc& s, int64_t r, int c)
{
    if (s.bf16) {
        const uint16_t b = static_cast<const uint16_t*>(s.data)[r * s.ld + c];
        return (double)__uint_as_float((uint32_t)b << 16);
    }
    return (double)static_cast<const float*>(s.data)[r * s.ld + c];
}

__global__ void __launch_bounds__(kStatThreads) k_colsum(ColSrc s, int64_t n, int cols,
                                                        const double* __restrict__ center,
                                                        int square, double* __restrict__ partial)
{
    __shared__ double acc[4][kMaxCols];
    const int c = threadIdx.x % kMaxCols, lane_row = threadIdx.x / kMaxCols;
    double a = 0.0;
    if (c < cols) {
        const double m = center ? center[c] : 0.0;
        for (int64_t r = (int64_t)blockIdx.x * 4 + lane_row; r < n; r += (int64_t)gridDim.x * 4) {
            const double v = col_value(s, r, c) - m;
            a += square ? v * v : v;
        }
    }
    acc[lane_row][c] = a;
    __syncthreads();
    if (lane_row == 0)
        partial[(int64_t)blockIdx.x * kMaxCols + c] =
            ((acc[0][c] + acc[1][c]) + acc[2][c]) + acc[3][c];
}

// Residual columns of the network: Y[r][c] - T[r][c] for c < cols, sums and
// sums of squares added into partial[block][0..63] and [64..127] (the same
// block layout chunk after chunk).
__global__ void __launch_bounds__(kStatThreads) k_resid(const float* __restrict__ Y, int64_t ldy,
                                                       const float* __restrict__ T, int64_t ldt,
                                                       int64_t n, int cols,
                                                       double* __restrict__ partial)
{
    __shared__ double acc[2][4][kMaxCols];
    const int c = threadIdx.x % kMaxCols, lane_row = threadIdx.x / kMaxCols;
    double a = 0.0, q = 0.0;
    if (c < cols) {
        for (int64_t r = (int64_t)blockIdx.x * 4 + lane_row; r < n; r += (int64_t)gridDim.x * 4) {
            const double v = (double)Y[r * ldy + c] - (double)T[r * ldt + c];
            a += v;
            q += v * v;
        }
    }
    acc[0][lane_row][c] = a;
    acc[1][lane_row][c] = q;
    __syncthreads();
    if (lane_row == 0) {
        double* p = partial + (int64_t)blockIdx.x * 2 * kMaxCols;
        p[c] += ((acc[0][0][c] + acc[0][1][c]) + acc[0][2][c]) + acc[0][3][c];
        p[kMaxCols + c] += ((acc[1][0][c] + acc[1][1][c]) + acc[1][2][c]) + acc[1][3][c];
    }
}

// Ordered sum of the block partials: out[c] = sum over blocks of
// partial[b][c] (width columns per block), one thread per column.
__global__ void k_partial_total(const double* __restrict__ partial, int blocks, int width,
                                double* __restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= width) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[(int64_t)b * width + c];
    out[c] = s;
}

__global__ void k_zero_f64(double* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

unsigned grid_for(int64_t work, int threads)
{
    const int64_t g = (work + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

extern "C" {

int adm1_gather_rows(const void* src, int64_t n_src, int64_t row_bytes, const int32_t* idx,
                     int64_t n_idx, void* dst, void* stream)
{
    if (!src || !idx || !dst) return ADM1_E_NULL;
    if (n_src < 0 || n_idx < 0 || row_bytes <= 0 || row_bytes % 4 != 0) return ADM1_E_SIZE;
    if (((uintptr_t)src & 3) || ((uintptr_t)dst & 3)) return ADM1_E_SIZE;
    if (!is_device(src) || !is_device(idx) || !is_device(dst)) return ADM1_E_NOT_DEVICE;
    if (n_idx == 0) return ADM1_OK;
    const int64_t words = row_bytes / 4;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n_idx * words, 256)), dim3(256), 0,
                       (hipStream_t)stream, static_cast<const uint32_t*>(src), n_src, words, idx,
                       n_idx, static_cast<uint32_t*>(dst));
    return hip_rc(hipGetLastError());
}

int adm1_permutation(int64_t n, uint64_t seed, int32_t* out, void* stream)
{
    if (!out) return ADM1_E_NULL;
    if (n < 0 || n > INT32_MAX) return ADM1_E_SIZE;
    if (!is_device(out)) return ADM1_E_NOT_DEVICE;
    if (n == 0) return ADM1_OK;
    Feistel f;
    int bits = 2;
    while (bits < 62 && ((uint64_t)1 << bits) < (uint64_t)n) bits += 2;
    f.half = bits / 2;
    f.mask = (uint32_t)(((uint64_t)1 << f.half) - 1);
    for (int k = 0; k < 4; ++k)
        f.keys[k] = mix32((uint32_t)(seed >> (16 * (k & 1))) ^ mix32((uint32_t)(seed >> 32) +
                                                                     0x9e3779b9u * (k + 1)));
    hipLaunchKernelGGL(k_permutation, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream,
                       f, n, out);
    return hip_rc(hipGetLastError());
}

int adm1_column_stats(const void* data, int32_t bf16, int64_t n, int32_t cols, int64_t ld,
                      double* mean_out, double* sd_out, void* stream)
{
    if (!data || !mean_out || !sd_out) return ADM1_E_NULL;
    if (n < 2 || cols < 1 || cols > kMaxCols || ld < cols || (bf16 != 0 && bf16 != 1))
        return ADM1_E_SIZE;
    if (!is_device(data)) return ADM1_E_NOT_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    double* buf = nullptr;  // partials [blocks][64], mean [64], second total [64]
    const size_t np = (size_t)kStatBlocks * kMaxCols;
    if (hipMalloc(&buf, (np + 2 * kMaxCols) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return ADM1_E_NOMEM;
    }
    double* mean = buf + np;
    double* tot2 = mean + kMaxCols;
    const ColSrc src{data, bf16, ld};
    int rc = ADM1_OK;
    double host[2][kMaxCols];
    hipLaunchKernelGGL(k_colsum, dim3(kStatBlocks), dim3(kStatThreads), 0, s, src, n, (int)cols,
                       (const double*)nullptr, 0, buf);
    hipLaunchKernelGGL(k_partial_total, dim3(1), dim3(kMaxCols), 0, s, buf, kStatBlocks,
                       kMaxCols, mean);
    rc = hip_rc(hipGetLastError());
    if (rc == ADM1_OK)
        rc = hip_rc(hipMemcpyAsync(host[0], mean, sizeof(host[0]), hipMemcpyDeviceToHost, s));
    if (rc == ADM1_OK) rc = hip_rc(hipStreamSynchronize(s));
    if (rc == ADM1_OK) {
        for (int c = 0; c < kMaxCols; ++c) host[0][c] = c < cols ? host[0][c] / (double)n : 0.0;
        rc = hip_rc(hipMemcpyAsync(mean, host[0], sizeof(host[0]), hipMemcpyHostToDevice, s));
    }
    if (rc == ADM1_OK) {
        hipLaunchKernelGGL(k_colsum, dim3(kStatBlocks), dim3(kStatThreads), 0, s, src, n,
                           (int)cols, (const double*)mean, 1, buf);
        hipLaunchKernelGGL(k_partial_total, dim3(1), dim3(kMaxCols), 0, s, buf, kStatBlocks,
                           kMaxCols, tot2);
        rc = hip_rc(hipGetLastError());
    }
    if (rc == ADM1_OK)
        rc = hip_rc(hipMemcpyAsync(host[1], tot2, sizeof(host[1]), hipMemcpyDeviceToHost, s));
    if (rc == ADM1_OK) rc = hip_rc(hipStreamSynchronize(s));
    if (rc == ADM1_OK)
        for (int c = 0; c < cols; ++c) {
            mean_out[c] = host[0][c];
            sd_out[c] = std::sqrt(host[1][c] / (double)(n - 1));
        }
    (void)hipFree(buf);
    return rc;
}

int adm1_surrogate_residual_stats(adm1_surrogate* sur, const uint16_t* X, const float* target,
                                  int64_t n, int64_t chunk, double* mean_out, double* msq_out,
                                  void* stream)
{
    if (!sur || !X || !target || !mean_out || !msq_out) return ADM1_E_NULL;
    if (n < 1 || chunk < 1) return ADM1_E_SIZE;
    if (!is_device(X) || !is_device(target)) return ADM1_E_NOT_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = chunk < n ? chunk : n;
    float* Y = nullptr;
    double* buf = nullptr;  // partials [blocks][128], totals [128]
    const size_t np = (size_t)kStatBlocks * 2 * kMaxCols;
    if (hipMalloc(&Y, (size_t)m * ADM1_MLP_OUT_LD * sizeof(float)) != hipSuccess ||
        hipMalloc(&buf, (np + 2 * kMaxCols) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        if (Y) (void)hipFree(Y);
        return ADM1_E_NOMEM;
    }
    double* tot = buf + np;
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for((int64_t)np, 256)), dim3(256), 0, s, buf,
                       (int64_t)np);
    int rc = hip_rc(hipGetLastError());
    for (int64_t a = 0; rc == ADM1_OK && a < n; a += m) {
        const int64_t rows = (n - a) < m ? (n - a) : m;
        rc = adm1_surrogate_forward(sur, X + a * ADM1_MLP_FEAT_LD, rows, Y, stream);
        if (rc == ADM1_OK) {
            hipLaunchKernelGGL(k_resid, dim3(kStatBlocks), dim3(kStatThreads), 0, s, Y,
                               (int64_t)ADM1_MLP_OUT_LD, target + a * ADM1_MLP_OUT,
                               (int64_t)ADM1_MLP_OUT, rows, ADM1_MLP_OUT, buf);
            rc = hip_rc(hipGetLastError());
        }
    }
    double host[2 * kMaxCols];
    if (rc == ADM1_OK) {
        hipLaunchKernelGGL(k_partial_total, dim3(1), dim3(2 * kMaxCols), 0, s, buf, kStatBlocks,
                           2 * kMaxCols, tot);
        rc = hip_rc(hipGetLastError());
    }
    if (rc == ADM1_OK)
        rc = hip_rc(hipMemcpyAsync(host, tot, sizeof(host), hipMemcpyDeviceToHost, s));
    if (rc == ADM1_OK) rc = hip_rc(hipStreamSynchronize(s));
    if (rc == ADM1_OK)
        for (int c = 0; c < ADM1_MLP_OUT; ++c) {
            mean_out[c] = host[c] / (double)n;
            msq_out[c] = host[kMaxCols + c] / (double)n;
        }
    (void)hipFree(Y);
    (void)hipFree(buf);
    return rc;
}

}  // extern "C"
