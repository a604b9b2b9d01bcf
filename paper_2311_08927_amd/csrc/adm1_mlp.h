// Surrogate MLP kernels: launchers and the padded parameter layout
// (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adm1 {

// Network 38 -> 256 -> 256 -> 256 -> 256 -> 35.  Inputs are padded to 64
// columns and outputs to 48 so every layer is a whole number of 16-wide
// matrix-core tiles; padded weights are held at zero by a mask.
constexpr int kMlpLayers = 5;
constexpr int kMlpIn = 38, kMlpHidden = 256, kMlpOut = 35;
constexpr int kMlpInPad = 64, kMlpOutPad = 48;
constexpr int kMlpDimIn[kMlpLayers] = {kMlpIn, kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden};
constexpr int kMlpDimOut[kMlpLayers] = {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden, kMlpOut};
constexpr int kMlpPadIn[kMlpLayers] = {kMlpInPad, kMlpHidden, kMlpHidden, kMlpHidden,
                                       kMlpHidden};
constexpr int kMlpPadOut[kMlpLayers] = {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden,
                                        kMlpOutPad};
// norm vector: in_mean[38], in_sd[38], out_mean[35], out_sd[35]
constexpr int kMlpNorm = 2 * kMlpIn + 2 * kMlpOut;

// Offsets of W_l ([in_pad][out_pad], row-major) and b_l ([out_pad]) in the
// flat padded FP32 parameter vector.
__host__ __device__ constexpr int64_t mlp_w_offset(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k)
        o += (int64_t)kMlpPadIn[k] * kMlpPadOut[k] + kMlpPadOut[k];
    return o;
}
__host__ __device__ constexpr int64_t mlp_b_offset(int l)
{
    return mlp_w_offset(l) + (int64_t)kMlpPadIn[l] * kMlpPadOut[l];
}
constexpr int64_t kMlpPadParams = mlp_w_offset(kMlpLayers);

// Device view of the network used by the forward kernel.
struct MlpDev {
    const uint16_t* WT[kMlpLayers];   // BF16 [out_pad][in_pad]
    const float* bias[kMlpLayers];    // FP32 [out_pad] (inside the master vector)
    float* z[4];                      // saved pre-activations [B][256] (training)
    uint16_t* hT[4];                  // saved activations, transposed [256][ldt] (training)
    uint16_t* xT;                     // saved input, transposed [64][ldt] (training)
    int64_t ldt;                      // row length of the transposed saves: B rounded up to 32
};

constexpr int kColsumChunks = 32;     // row chunks of the bias-gradient column sums

hipError_t mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, float* Y, bool save,
                       hipStream_t s);
// C[m][n] = sum_k A[m lda + k] B[n ldb + k]; K % 16 == 0, lda and ldb
// multiples of 8; with splitk > 1 the partials (splitk M ldc floats) go
// through `partial` and are added in fixed order.
hipError_t gemm_tn(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, float* C,
                   int64_t ldc, int M, int N, int K, int splitk, float* partial, hipStream_t s);
hipError_t mlp_loss(const float* Y, const float* T, int64_t B, int64_t ldt, float* dY,
                    uint16_t* dYb, uint16_t* dYT, float* partial, float* loss, hipStream_t s);
hipError_t gelu_bwd(const float* dH, const float* Z, int64_t B, int64_t ldt, float* dZ,
                    uint16_t* dZb, uint16_t* dZT, hipStream_t s);
// part: kColsumChunks * cols floats of scratch
hipError_t colsum(const float* M, int64_t rows, int ld, int cols, float* out, float* part,
                  hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, const uint8_t* mask, int64_t cnt,
                float lr, float b1, float b2, float eps, int step, hipStream_t s);
hipError_t pack(const float* W, int in, int out, uint16_t* WT, uint16_t* Wb, hipStream_t s);
hipError_t featurize(const double* state, int64_t ld, const double* T, const double* D,
                     double dt, int64_t n, const float* norm, const double* floor_,
                     uint16_t* X, hipStream_t s);
hipError_t targets(const double* x0, const double* x1, int64_t ld, int64_t n, const float* norm,
                   const double* floor_, float* Tg, hipStream_t s);

}  // namespace adm1
