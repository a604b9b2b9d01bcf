// Learned surrogate of the per-particle ADM1 step: an MLP that maps the
// log-scaled state, temperature, interval and feed flag of a particle to
// the log-space increments of its 35 entries over one coupling interval.
//
// Network 38 -> 256 -> 256 -> 256 -> 256 -> 35, GELU (erf form), BF16
// weights and activations, FP32 accumulation on the matrix cores, FP32
// master weights and Adam.
//
// Kernels:
//   k_mlp_fwd    fused forward (v_mfma_f32_16x16x32_bf16): a 64-row tile
//                stays in LDS for all five layers (two 64 x 264 BF16
//                buffers), weights stream from L2 in the transposed layout
//                WT[out][in] so each lane's eight k-values are one 16-byte
//                load; optional saving of pre-activations (FP32) and
//                activations (BF16) for the backward pass;
//   k_gemm_tn    BF16 GEMM with both operands contiguous along the
//                contraction (v_mfma_f32_16x16x32_bf16, register-tiled,
//                split-K): the backward pass dH = dZ W^T and dW = H^T dZ on
//                the transposed copies the forward and backward kernels save;
//   k_loss, k_gelu_bwd, k_colsum, k_splitk_sum, k_adam, k_pack: the
//                elementwise and reduction steps of training;
//   k_featurize  the network input from the FP64 state.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "adm1_mlp.h"

namespace adm1 {
namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t f2bf(float x)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t q = (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    return (uint16_t)(((u & 0x7f800000u) == 0x7f800000u) ? q : r);
}
__device__ __forceinline__ float bf2f(uint16_t b)
{
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ f32x4 mfma16(s16x4 a, s16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// GELU with a branch-free erf: Abramowitz & Stegun, Handbook of
// Mathematical Functions, eq. 7.1.26 (|error| <= 1.5e-7 on the real line),
// erf(x) = 1 - P(t) exp(-x^2), t = 1 / (1 + p x), x >= 0, odd extension.
// Rearranged as z Phi(z) = (z + |z|) / 2 - |z| t q(t) exp(-z^2 / 2), with
// q = P / (2 t) (coefficients halved) and p / sqrt(2) folded into t: two
// transcendentals and eleven other operations.
__device__ __forceinline__ float gelu_fast(float z)
{
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
    const float q =
        0.127414796f + t * (-0.142248368f + t * (0.7107068705f + t * (-0.7265760135f +
                                                                     t * 0.5307027145f)));
    // exp(-z^2/2) = 2^(-(z k)^2), k = sqrt(log2(e) / 2)
    const float y = z * 0.84932180028801904f;
    const float e = __builtin_amdgcn_exp2f(-(y * y));
    return fmaf(-q, az * t * e, 0.5f * (z + az));
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values to packed BF16 with the hardware conversion (round to
// nearest even, NaN stays NaN), low half first.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2 v = __builtin_convertvector(f32x2{lo, hi}, bf16x2);
    return __builtin_bit_cast(uint32_t, v);
}

// ---------------------------------------------------------------------------
// Fused forward on gfx950's 16x16x32 BF16 MFMA.  Operand layout (lane l):
//   A (16 x 32, rows i, k):  row l % 16, k = 8 (l / 16) + t, t = 0..7
//   B (32 x 16, k, cols j):  col l % 16, k = 8 (l / 16) + t
//   C (16 x 16):             col l % 16, rows 4 (l / 16) + t, t = 0..3
// Each layer is computed transposed, Z^T = W^T H^T: A is a 16-feature slice
// of W^T (eight contiguous k-values per lane: one 16-byte load), B a
// 16-row slice of the activations (one 16-byte LDS read), and each lane's
// four results are four consecutive features of one row, stored as one
// 8-byte LDS write (16 bytes for FP32 outputs).
// A block of 256 threads owns 64 rows; the activations of all five layers
// stay in two 64 x 264 BF16 LDS buffers (67.6 KB: two blocks per CU).
// Wave w owns the feature tiles [w CTW, (w + 1) CTW) of a layer: it holds
// their weight fragments for every k-step in registers (requested while the
// previous layer finishes), then runs the four 16-row tiles one after the
// other; a tile's epilogue
// (bias, GELU, BF16 packing) is plain straight-line VALU work that the
// scheduler interleaves with the next tile's matrix instructions.  The
// per-particle GELU work (1,024 evaluations) costs more VALU cycles than
// the 215,296 MACs cost matrix-core cycles, so this overlap bounds the
// kernel.
// ---------------------------------------------------------------------------
constexpr int TM = 64;       // rows per block
constexpr int RT = TM / 16;  // row tiles
constexpr int LDH = 264;     // LDS row stride (BF16 elements): 528 B, 16-byte aligned
constexpr int kFwdWaves = 8;     // forward: waves per block
constexpr int kFwdThreads = 64 * kFwdWaves;

struct FwdArgs {
    const uint16_t* X;   // [n][64] BF16
    int64_t n;
    const uint16_t* WT[5];
    const float* b[5];
    float* Y;            // [n][48] FP32
    float* zsave[4];     // [n][256] FP32 pre-activations (with SAVE)
    uint16_t* hT[4];     // [256][ldt] BF16 activations, transposed (with SAVE)
    uint16_t* xT;        // [64][ldt] BF16 input, transposed (with SAVE)
    int64_t ldt;         // row length of the transposed saves, >= n
};

// A wave's weight fragments and biases for one layer: feature tiles
// [c0, c0 + CTW) of W^T, every k-step.
template <int K, int NOUT>
struct LayerW {
    static constexpr int CT = NOUT / 16;          // feature tiles
    static constexpr int CTW = (CT + kFwdWaves - 1) / kFwdWaves;  // per wave
    static constexpr int KS = K / 32;             // k-steps
    s16x8 wf[CTW][KS];
    f32x4 bc[CTW];
};

// Issue order = use order (bias, then k-step by k-step), so the first matrix
// instructions wait only for the first loads (the memory counter retires
// loads in order).  Tiles past the layer's width (the idle wave of the
// narrow last layer) load the last tile again: no branch, and their results
// are never stored.
template <int K, int NOUT>
__device__ __forceinline__ void load_layer(const FwdArgs& a, int layer, LayerW<K, NOUT>& w)
{
    using L = LayerW<K, NOUT>;
    const int lane = threadIdx.x & 63, c0 = (threadIdx.x >> 6) * L::CTW;
    const int kq = 8 * (lane >> 4), li = lane & 15, fq = 4 * (lane >> 4);
    const uint16_t* WT = a.WT[layer];
    int ct[L::CTW];
#pragma unroll
    for (int c = 0; c < L::CTW; ++c) ct[c] = c0 + c < L::CT ? c0 + c : L::CT - 1;
#pragma unroll
    for (int c = 0; c < L::CTW; ++c) w.bc[c] = *(const f32x4*)(a.b[layer] + ct[c] * 16 + fq);
#pragma unroll
    for (int ks = 0; ks < L::KS; ++ks)
#pragma unroll
        for (int c = 0; c < L::CTW; ++c)
            w.wf[c][ks] = *(const s16x8*)(WT + (int64_t)(ct[c] * 16 + li) * K + ks * 32 + kq);
}

// One layer: out[TM][NOUT] = act(in[TM][K] W + b) with the weights in `w`.
// Once the last tile's matrix instructions are issued, the next layer's
// weights are requested into `next` (layer + 1), so their latency overlaps
// the last epilogue and the barrier.  SAVE also writes the pre-activations
// and activations of rows < n for the backward pass.
template <int K, int NOUT, bool LAST, bool SAVE, int NK, int NNOUT>
__device__ __forceinline__ void fwd_layer(const FwdArgs& a, int layer, const LayerW<K, NOUT>& w,
                                          LayerW<NK, NNOUT>& next, const uint16_t* in,
                                          uint16_t* out, int64_t row0)
{
    using L = LayerW<K, NOUT>;
    constexpr int CT = L::CT, CTW = L::CTW, KS = L::KS;
    const int lane = threadIdx.x & 63, c0 = (threadIdx.x >> 6) * CTW;
    const int kq = 8 * (lane >> 4), li = lane & 15, fq = 4 * (lane >> 4);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        f32x4 acc[CTW];
#pragma unroll
        for (int c = 0; c < CTW; ++c) acc[c] = w.bc[c];
        // the idle waves of the narrow last layer skip its matrix work
        if (!LAST || c0 < CT) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const s16x8 hf = *(const s16x8*)(in + (r * 16 + li) * LDH + ks * 32 + kq);
#pragma unroll
                for (int c = 0; c < CTW; ++c) acc[c] = mfma32(w.wf[c][ks], hf, acc[c]);
            }
        }
        if (!LAST && r == RT - 1) load_layer<NK, NNOUT>(a, layer + 1, next);
        if (c0 >= CT) continue;
        const int row = r * 16 + li;
        const int64_t grow = row0 + row;
#pragma unroll
        for (int c = 0; c < CTW; ++c) {
            if (c0 + c >= CT) continue;
            const int f = (c0 + c) * 16 + fq;  // first of this lane's four features
            const f32x4 z = acc[c];
            if (LAST) {
                if (grow < a.n) *(f32x4*)(a.Y + grow * 48 + f) = z;
            } else {
                uint2 hb;
                hb.x = pack_bf16(gelu_fast(z[0]), gelu_fast(z[1]));
                hb.y = pack_bf16(gelu_fast(z[2]), gelu_fast(z[3]));
                *(uint2*)(out + row * LDH + f) = hb;
                if (SAVE && grow < a.n) *(f32x4*)(a.zsave[layer] + grow * 256 + f) = z;
                if (SAVE && grow < a.ldt) {
                    uint16_t* ht = a.hT[layer] + (int64_t)f * a.ldt + grow;
                    ht[0] = (uint16_t)hb.x;
                    ht[a.ldt] = (uint16_t)(hb.x >> 16);
                    ht[2 * a.ldt] = (uint16_t)hb.y;
                    ht[3 * a.ldt] = (uint16_t)(hb.y >> 16);
                }
            }
        }
    }
}

template <bool SAVE>
__global__ void __launch_bounds__(kFwdThreads, 2) k_mlp_fwd(FwdArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t buf0[TM * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t buf1[TM * LDH];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    LayerW<64, 256> w0;
    LayerW<256, 256> wa, wb;
    LayerW<256, 48> w4;
    load_layer<64, 256>(a, 0, w0);
    // input tile: 64 rows x 64 features, 16 bytes per load
    for (int e = threadIdx.x; e < TM * 8; e += kFwdThreads) {
        const int row = e >> 3, q = (e & 7) * 8;
        const int64_t grow = row0 + row;
        s16x8 v = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (grow < a.n) v = *(const s16x8*)(a.X + grow * 64 + q);
        *(s16x8*)(buf0 + row * LDH + q) = v;
        if (SAVE && grow < a.ldt) {
#pragma unroll
            for (int t = 0; t < 8; ++t) a.xT[(int64_t)(q + t) * a.ldt + grow] = (uint16_t)v[t];
        }
    }
    __syncthreads();
    fwd_layer<64, 256, false, SAVE>(a, 0, w0, wa, buf0, buf1, row0);
    __syncthreads();
    fwd_layer<256, 256, false, SAVE>(a, 1, wa, wb, buf1, buf0, row0);
    __syncthreads();
    fwd_layer<256, 256, false, SAVE>(a, 2, wb, wa, buf0, buf1, row0);
    __syncthreads();
    fwd_layer<256, 256, false, SAVE>(a, 3, wa, w4, buf1, buf0, row0);
    __syncthreads();
    fwd_layer<256, 48, true, SAVE>(a, 4, w4, w4, buf0, buf1, row0);
}

// ---------------------------------------------------------------------------
// Backward GEMM, both operands contiguous along the contraction index:
//   C[m][n] (+ z splitc) = sum_{k in chunk z} A[m lda + k] B[n ldb + k]
// (BF16 in, FP32 out).  dW = H^T dZ reads the transposed activations and
// gradients the forward and backward kernels save; dH = dZ W^T reads dZ
// and W[in][out] as stored.  Each wave owns a (16 kTnRows) x 64 block of C
// (kTnRows x 4 tiles of 16 x 16) and loads its operand fragments straight
// from memory (16 bytes per lane, three k-steps in flight); a block is
// 2 x 2 waves.  These products are small (~1 GFLOP), so the tile is sized
// for enough waves to fill the chip rather than for maximal reuse.  K is a
// multiple of 16: a remainder of 16 runs on the 16x16x16 instruction.
// Rows and columns past M and N load the last valid ones and are not stored.
// ---------------------------------------------------------------------------
struct TnArgs {
    const uint16_t* A;
    int64_t lda;
    const uint16_t* B;
    int64_t ldb;
    float* C;
    int64_t ldc, splitc;
    int M, N, K, kchunk;
};

constexpr int kTnRows = 2;  // 16-row tiles per wave (a wave owns 16 kTnRows x 64 of C)

__global__ void __launch_bounds__(256) k_gemm_tn(TnArgs g)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.y * (2 * 16 * kTnRows) + (w & 1) * (16 * kTnRows);
    const int n0 = blockIdx.x * 128 + (w >> 1) * 64;
    if (m0 >= g.M || n0 >= g.N) return;  // no barriers below: a wave may leave
    const int kb = blockIdx.z * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    const int li = lane & 15, q = lane >> 4;
    const uint16_t* ap[kTnRows];
    const uint16_t* bp[4];
#pragma unroll
    for (int t = 0; t < kTnRows; ++t)
        ap[t] = g.A + (int64_t)min(m0 + 16 * t + li, g.M - 1) * g.lda;
#pragma unroll
    for (int t = 0; t < 4; ++t) bp[t] = g.B + (int64_t)min(n0 + 16 * t + li, g.N - 1) * g.ldb;
    f32x4 acc[kTnRows][4];
#pragma unroll
    for (int r = 0; r < kTnRows; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kfull = kb + ((ke - kb) / 32) * 32;
    // three k-steps of fragments in flight (a ring of register buffers):
    // a step's loads are issued two steps before its matrix instructions
    s16x8 fa[3][kTnRows], fb[3][4];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (kb + 32 * j < kfull) {
#pragma unroll
            for (int t = 0; t < kTnRows; ++t) fa[j][t] = *(const s16x8*)(ap[t] + kb + 32 * j + 8 * q);
#pragma unroll
            for (int t = 0; t < 4; ++t) fb[j][t] = *(const s16x8*)(bp[t] + kb + 32 * j + 8 * q);
        }
    for (int k = kb; k < kfull; k += 96) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int kj = k + 32 * j;
            if (kj < kfull) {
#pragma unroll
                for (int r = 0; r < kTnRows; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[r][c] = mfma32(fa[j][r], fb[j][c], acc[r][c]);
                if (kj + 96 < kfull) {
#pragma unroll
                    for (int t = 0; t < kTnRows; ++t)
                        fa[j][t] = *(const s16x8*)(ap[t] + kj + 96 + 8 * q);
#pragma unroll
                    for (int t = 0; t < 4; ++t) fb[j][t] = *(const s16x8*)(bp[t] + kj + 96 + 8 * q);
                }
            }
        }
    }
    if (kfull < ke) {  // 16 left
        s16x4 a4[kTnRows], b4[4];
#pragma unroll
        for (int t = 0; t < kTnRows; ++t) a4[t] = *(const s16x4*)(ap[t] + kfull + 4 * q);
#pragma unroll
        for (int t = 0; t < 4; ++t) b4[t] = *(const s16x4*)(bp[t] + kfull + 4 * q);
#pragma unroll
        for (int r = 0; r < kTnRows; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = mfma16(a4[r], b4[c], acc[r][c]);
    }
    float* C = g.C + (int64_t)blockIdx.z * g.splitc;
#pragma unroll
    for (int r = 0; r < kTnRows; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = n0 + 16 * c + li;
            if (col >= g.N) continue;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = m0 + 16 * r + 4 * q + t;
                if (row < g.M) C[(int64_t)row * g.ldc + col] = acc[r][c][t];
            }
        }
}

// Sum of split-K partials in fixed order: out[i] = sum_z part[z * stride + i].
__global__ void k_splitk_sum(const float* part, int64_t stride, int S, int64_t cnt, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    // four running sums (z mod 4), added in a fixed order: independent loads
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    int z = 0;
    for (; z + 4 <= S; z += 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += part[(int64_t)(z + j) * stride + i];
    }
    for (; z < S; ++z) s[0] += part[(int64_t)z * stride + i];
    out[i] = (s[0] + s[1]) + (s[2] + s[3]);
}

// MSE loss on the 35 outputs: dY = 2 (Y - T) / (B 35) as FP32 [B][48], BF16
// [B][48] and BF16 transposed [48][ldt] (zero in rows b >= B), and
// per-block partial sums of the squared error.  A thread owns eight
// consecutive rows of one column, so the transposed copy is one 16-byte
// store.
__global__ void __launch_bounds__(256) k_loss(const float* Y, const float* T, int64_t B,
                                              int64_t ldt, float* dY, uint16_t* dYb,
                                              uint16_t* dYT, float* partial)
{
    __shared__ float red[256];
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b8 = gid / 48;
    const int c = (int)(gid - b8 * 48);
    float s = 0.f;
    if (b8 * 8 < ldt) {
        s16x8 t8;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t r = b8 * 8 + t;
            float g = 0.f;
            if (r < B) {
                if (c < 35) {
                    const float d = Y[r * 48 + c] - T[r * 35 + c];
                    s += d * d;
                    g = 2.f * d / (float)(B * 35);
                }
                dY[r * 48 + c] = g;
                dYb[r * 48 + c] = f2bf(g);
            }
            t8[t] = (short)f2bf(g);
        }
        *(s16x8*)(dYT + (int64_t)c * ldt + b8 * 8) = t8;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_final(const float* partial, int nb, int64_t B,
                                                    float* loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int k = threadIdx.x; k < nb; k += 256) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)(B * 35);
}

// dZ = dH * GELU'(Z) for a [B][256] layer: FP32 and BF16 [B][256] and BF16
// transposed [256][ldt] (zero in rows b >= B).  A thread owns eight
// consecutive rows of one column.
__global__ void __launch_bounds__(256) k_gelu_bwd(const float* dH, const float* Z, int64_t B,
                                                  int64_t ldt, float* dZ, uint16_t* dZb,
                                                  uint16_t* dZT)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b8 = gid >> 8;
    const int c = (int)(gid & 255);
    if (b8 * 8 >= ldt) return;
    s16x8 t8;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t r = b8 * 8 + t;
        uint16_t hb = 0;
        if (r < B) {
            const float g = dH[r * 256 + c] * gelu_grad(Z[r * 256 + c]);
            hb = f2bf(g);
            dZ[r * 256 + c] = g;
            dZb[r * 256 + c] = hb;
        }
        t8[t] = (short)hb;
    }
    *(s16x8*)(dZT + (int64_t)c * ldt + b8 * 8) = t8;
}

// Column sums in fixed order, first stage: part[z][c] = sum of M[r][c] over
// the rows of chunk z (64 columns per block, four row phases per column,
// coalesced 256-byte row reads); k_splitk_sum adds the chunks in order.
__global__ void __launch_bounds__(256) k_colsum(const float* M, int64_t rows, int ld, int cols,
                                                int64_t chunk, float* part)
{
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * chunk;
    const int64_t r1 = min(rows, r0 + chunk);
    // eight running sums per thread (rows r0 + ph + 4 j, j mod 8), added in
    // a fixed order: independent loads stay in flight
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (c < cols) {
        int64_t r = r0 + ph;
        for (; r + 28 < r1; r += 32) {
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += M[(r + 4 * j) * ld + c];
        }
        for (; r < r1; r += 4) acc[0] += M[r * ld + c];
    }
    const float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    red[ph][cl] = s;
    __syncthreads();
    if (ph == 0 && c < cols)
        part[(int64_t)blockIdx.y * cols + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) +
                                               red[3][cl];
}

// Adam on the FP32 master parameters (padded entries carry a zero mask).
__global__ void k_adam(float* p, const float* g, float* m, float* v, const uint8_t* mask,
                       int64_t cnt, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    if (!mask[i]) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 working copies of one layer from the FP32 master W[in][out]:
// WT[out][in] (forward) and W[in][out] (backward).
__global__ void k_pack(const float* W, int in, int out, uint16_t* WT, uint16_t* Wb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)in * out) return;
    const int r = (int)(i / out), c = (int)(i - (int64_t)r * out);
    const uint16_t b = f2bf(W[i]);
    Wb[i] = b;
    WT[(int64_t)c * in + r] = b;
}

// Natural logarithm for the features, x > 0: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.172,
// summed to the s^15 term (Abramowitz & Stegun, Handbook of Mathematical
// Functions, eq. 4.1.27); the first omitted term is below 1.2e-14, far under
// the FP32 rounding the features receive.  About half the operations of the
// library's double-precision log, short enough to inline 35 times.  +inf
// and NaN are returned unchanged.
__device__ __forceinline__ double log_feature(double x)
{
    if (!(x < INFINITY)) return x;
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        --e;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    const double p =
        1.0 / 3 + s2 * (1.0 / 5 + s2 * (1.0 / 7 + s2 * (1.0 / 9 + s2 * (1.0 / 11 + s2 * (1.0 / 13 +
                                                                                   s2 / 15)))));
    const double two_s = 2.0 * s;
    const double lm = fma(two_s * s2, p, two_s);
    // e ln 2 with ln 2 split so e * ln2_hi is exact (|e| < 2^11)
    const double de = (double)e;
    return fma(de, 0.693147180559945309417232121458 - 0.693145751953125, lm) +
           de * 0.693145751953125;
}

// Network input from the FP64 state: log(max(x, floor)) of the 35 entries,
// temperature, log dt and the feed flag, standardised; BF16 [n][64].
__global__ void __launch_bounds__(256) k_featurize(const double* state, int64_t ld,
                                                   const double* T, const double* D, double dt,
                                                   int64_t n, const float* norm,
                                                   const double* floor_, uint16_t* X)
{
    // a block's 256 rows are contiguous in X: they are assembled in LDS
    // (row stride 9 x 16 bytes, against bank conflicts) and written as
    // consecutive 16-byte stores instead of one scattered row per thread
    __shared__ s16x8 tile[256 * 9];
    const int64_t row0 = (int64_t)blockIdx.x * 256;
    const int64_t i = row0 + threadIdx.x;
    const float* mean = norm;
    const float* sd = norm + 38;
    if (i < n) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s16x8 v;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = q * 8 + t;
                float f = 0.0f;
                if (k < 35) {
                    const double x = fmax(state[k * ld + i], floor_[k]);
                    f = ((float)log_feature(x) - mean[k]) / sd[k];
                } else if (k == 35) {
                    f = ((float)T[i] - mean[35]) / sd[35];
                } else if (k == 36) {
                    f = ((float)log(dt) - mean[36]) / sd[36];
                } else if (k == 37) {
                    f = ((D[i] > 0.0 ? 1.f : 0.f) - mean[37]) / sd[37];
                }
                v[t] = (short)(k < 38 ? f2bf(f) : 0);
            }
            tile[threadIdx.x * 9 + q] = v;
        }
    }
    __syncthreads();
    const int64_t rows = n - row0 < 256 ? n - row0 : 256;
    s16x8* xo = (s16x8*)(X + row0 * 64);
    for (int c = threadIdx.x; c < rows * 8; c += 256) xo[c] = tile[(c >> 3) * 9 + (c & 7)];
}

// Training targets: standardised increments of log(max(x, floor)).
__global__ void __launch_bounds__(256) k_targets(const double* x0, const double* x1,
                                                 int64_t ld, int64_t n, const float* norm,
                                                 const double* floor_, float* Tg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* mean = norm + 76;
    const float* sd = norm + 111;
    for (int k = 0; k < 35; ++k) {
        const double a = fmax(x0[k * ld + i], floor_[k]), b = fmax(x1[k * ld + i], floor_[k]);
        Tg[i * 35 + k] = ((float)(log(b) - log(a)) - mean[k]) / sd[k];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, float* Y, bool save,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    FwdArgs a;
    a.X = X;
    a.n = n;
    for (int l = 0; l < 5; ++l) {
        a.WT[l] = m.WT[l];
        a.b[l] = m.bias[l];
    }
    a.Y = Y;
    for (int l = 0; l < 4; ++l) {
        a.zsave[l] = save ? m.z[l] : nullptr;
        a.hT[l] = save ? m.hT[l] : nullptr;
    }
    a.xT = save ? m.xT : nullptr;
    a.ldt = save ? m.ldt : 0;
    const unsigned grid = (unsigned)((n + TM - 1) / TM);
    if (save)
        hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(grid), dim3(kFwdThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_mlp_fwd<false>, dim3(grid), dim3(kFwdThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t gemm_tn(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, float* C,
                   int64_t ldc, int M, int N, int K, int splitk, float* partial, hipStream_t s)
{
    if (M <= 0 || N <= 0 || K <= 0 || K % 16 != 0 || lda % 8 != 0 || ldb % 8 != 0)
        return hipErrorInvalidValue;
    TnArgs g;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.M = M; g.N = N; g.K = K;
    const int bm = 2 * 16 * kTnRows;
    const dim3 tiles((unsigned)((N + 127) / 128), (unsigned)((M + bm - 1) / bm));
    if (splitk <= 1) {
        g.C = C; g.ldc = ldc; g.splitc = 0; g.kchunk = K;
        hipLaunchKernelGGL(k_gemm_tn, dim3(tiles.x, tiles.y, 1), dim3(256), 0, s, g);
        return hipGetLastError();
    }
    const int kchunk = ((K + splitk - 1) / splitk + 31) / 32 * 32;
    const int S = (K + kchunk - 1) / kchunk;
    g.C = partial; g.ldc = ldc; g.splitc = (int64_t)M * ldc; g.kchunk = kchunk;
    hipLaunchKernelGGL(k_gemm_tn, dim3(tiles.x, tiles.y, S), dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t cnt = (int64_t)M * ldc;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       partial, cnt, S, cnt, C);
    return hipGetLastError();
}

hipError_t mlp_loss(const float* Y, const float* T, int64_t B, int64_t ldt, float* dY,
                    uint16_t* dYb, uint16_t* dYT, float* partial, float* loss, hipStream_t s)
{
    const int nb = (int)((ldt / 8 * 48 + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, Y, T, B, ldt, dY, dYb, dYT, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, partial, nb, B, loss);
    return hipGetLastError();
}

hipError_t gelu_bwd(const float* dH, const float* Z, int64_t B, int64_t ldt, float* dZ,
                    uint16_t* dZb, uint16_t* dZT, hipStream_t s)
{
    const int64_t threads = ldt / 8 * 256;
    hipLaunchKernelGGL(k_gelu_bwd, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, dH,
                       Z, B, ldt, dZ, dZb, dZT);
    return hipGetLastError();
}

hipError_t colsum(const float* M, int64_t rows, int ld, int cols, float* out, float* part,
                  hipStream_t s)
{
    const int64_t nz = std::min<int64_t>(kColsumChunks, std::max<int64_t>(1, rows / 256));
    const int64_t chunk = (rows + nz - 1) / nz;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((cols + 63) / 64), (unsigned)nz), dim3(256), 0,
                       s, M, rows, ld, cols, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, part,
                       (int64_t)cols, (int)nz, (int64_t)cols, out);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* mo, float* v, const uint8_t* mask, int64_t cnt,
                float lr, float b1, float b2, float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, g, mo,
                       v, mask, cnt, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t pack(const float* W, int in, int out, uint16_t* WT, uint16_t* Wb, hipStream_t s)
{
    const int64_t cnt = (int64_t)in * out;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, W, in, out,
                       WT, Wb);
    return hipGetLastError();
}

hipError_t featurize(const double* state, int64_t ld, const double* T, const double* D,
                     double dt, int64_t n, const float* norm, const double* floor_,
                     uint16_t* X, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_featurize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, state,
                       ld, T, D, dt, n, norm, floor_, X);
    return hipGetLastError();
}

hipError_t targets(const double* x0, const double* x1, int64_t ld, int64_t n, const float* norm,
                   const double* floor_, float* Tg, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x0, x1,
                       ld, n, norm, floor_, Tg);
    return hipGetLastError();
}

}  // namespace adm1
