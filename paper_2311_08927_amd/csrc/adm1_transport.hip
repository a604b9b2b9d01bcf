// Coupling-driver kernels: Lagrangian displacement of the particles between
// coupling steps and the inlet feed mask.
//
// In the paper the particle motion comes from the SPH solver (sec. 2.3: each
// AD particle follows its SPH particle; advection needs no transport term).
// Here a smooth, divergence-free analytic field stands in for it in a
// cylindrical tank of radius R and height H: solid-body rotation Omega plus
// axisymmetric Stokes stream-function modes
//     psi(r, z) = sum_k a_k r^2 (R^2 - r^2) sin(k pi z / H),
//     u_r = -(1/r) dpsi/dz,  u_z = (1/r) dpsi/dr,  u_theta = Omega r,
// which is tangent to the wall and to the bottom and top.  Positions are
// FP32 structure-of-arrays pos[3][ld] (x, y, z in m).  The meridional part
// (u_r, u_z) is axisymmetric and so commutes with the rotation: each substep
// is a classical RK4 step of the meridional flow followed by the exact turn
// of the (x, y) plane by Omega h (RK4 on the rotation itself would shrink
// every orbit by about 2 % per 1 s substep at 12 rpm).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "adm1.h"

namespace adm1 {
namespace {

struct Field {
    float cos_wh, sin_wh;  // turn of one substep
    float R, H;
    float kz;              // pi / H
    // per mode k (1-based): a_k (axial) and a_k k pi / H (radial), so the
    // velocity is u_r/r = -(R^2 - r^2) sum_k rad_k cos(k kz z),
    // u_z = (2 R^2 - 4 r^2) sum_k ax_k sin(k kz z)
    float ax[ADM1_FLOW_MODES];
    float rad[ADM1_FLOW_MODES];
};

// Meridional velocity (the rotation is applied exactly, outside RK4) of NM
// modes.  sin and cos of k kz z come from those of kz z by angle addition:
// one transcendental evaluation per velocity, on the hardware sine/cosine
// (argument in [0, pi]).
template <int NM>
__device__ __forceinline__ void velocity(const Field& F, float x, float y, float z, float& ux,
                                         float& uy, float& uz)
{
    const float r2 = x * x + y * y;
    const float R2 = F.R * F.R;
    float s1 = 0.0f, c1 = 1.0f;
    if (NM > 0) __sincosf(F.kz * z, &s1, &c1);
    float s = s1, c = c1, sc = 0.0f, ss = 0.0f;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        sc = fmaf(F.rad[k], c, sc);
        ss = fmaf(F.ax[k], s, ss);
        const float sn = fmaf(s, c1, c * s1);
        c = fmaf(c, c1, -s * s1);
        s = sn;
    }
    const float radial = -(R2 - r2) * sc;  // u_r / r
    ux = radial * x;
    uy = radial * y;
    uz = (2.0f * R2 - 4.0f * r2) * ss;
}

__device__ __forceinline__ void clamp_tank(const Field& F, float& x, float& y, float& z)
{
    const float r2 = x * x + y * y;
    if (r2 > F.R * F.R) {
        const float s = F.R * rsqrtf(r2);
        x *= s;
        y *= s;
    }
    z = fminf(fmaxf(z, 0.0f), F.H);
}

template <int NM>
__global__ void __launch_bounds__(256) k_advect(float* pos, int64_t ld, int64_t n, Field F,
                                                float h, int nsub)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = pos[i], y = pos[ld + i], z = pos[2 * ld + i];
    for (int s = 0; s < nsub; ++s) {
        float k1x, k1y, k1z, k2x, k2y, k2z, k3x, k3y, k3z, k4x, k4y, k4z;
        velocity<NM>(F, x, y, z, k1x, k1y, k1z);
        velocity<NM>(F, x + 0.5f * h * k1x, y + 0.5f * h * k1y, z + 0.5f * h * k1z, k2x, k2y, k2z);
        velocity<NM>(F, x + 0.5f * h * k2x, y + 0.5f * h * k2y, z + 0.5f * h * k2z, k3x, k3y, k3z);
        velocity<NM>(F, x + h * k3x, y + h * k3y, z + h * k3z, k4x, k4y, k4z);
        x += h * (1.0f / 6.0f) * (k1x + 2.0f * k2x + 2.0f * k3x + k4x);
        y += h * (1.0f / 6.0f) * (k1y + 2.0f * k2y + 2.0f * k3y + k4y);
        z += h * (1.0f / 6.0f) * (k1z + 2.0f * k2z + 2.0f * k3z + k4z);
        const float xr = F.cos_wh * x - F.sin_wh * y;
        y = F.sin_wh * x + F.cos_wh * y;
        x = xr;
        clamp_tank(F, x, y, z);
    }
    pos[i] = x;
    pos[ld + i] = y;
    pos[2 * ld + i] = z;
}

// Inlet membership at the start of the interval: z >= z_min and r <= r_max.
__global__ void __launch_bounds__(256) k_feed_mask(const float* pos, int64_t ld, int64_t n,
                                                   float z_min, float r_max, double D_zone,
                                                   int32_t fidx_zone, int32_t fidx_out,
                                                   double* D, int32_t* fidx, uint8_t* flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = pos[i], y = pos[ld + i], z = pos[2 * ld + i];
    const bool in = z >= z_min && x * x + y * y <= r_max * r_max;
    D[i] = in ? D_zone : 0.0;
    fidx[i] = in ? fidx_zone : fidx_out;
    if (flag) flag[i] = in ? 1 : 0;
}

bool is_dev(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
           at.type == hipMemoryTypeUnified;
}

}  // namespace
}  // namespace adm1

extern "C" {

int adm1_advect(float* pos, int64_t ld, int64_t n, const adm1_flow* flow, double dt_seconds,
                int32_t substeps, void* stream)
{
    if (!pos || !flow) return ADM1_E_NULL;
    if (n < 0 || ld < n || ld <= 0 || ld % 64 != 0) return ADM1_E_SIZE;
    if (!(dt_seconds > 0.0) || substeps < 1) return ADM1_E_DT;
    if (flow->nmodes < 0 || flow->nmodes > ADM1_FLOW_MODES || !(flow->R > 0.0) ||
        !(flow->H > 0.0))
        return ADM1_E_OPTS;
    if (!adm1::is_dev(pos)) return ADM1_E_NOT_DEVICE;
    if (n == 0) return ADM1_OK;
    adm1::Field F;
    const double wh = flow->omega * (dt_seconds / substeps);
    F.cos_wh = (float)std::cos(wh);
    F.sin_wh = (float)std::sin(wh);
    F.R = (float)flow->R;
    F.H = (float)flow->H;
    const double kz = 3.14159265358979323846 / flow->H;
    F.kz = (float)kz;
    for (int k = 0; k < ADM1_FLOW_MODES; ++k) {
        const double a = k < flow->nmodes ? flow->a[k] : 0.0;
        F.ax[k] = (float)a;
        F.rad[k] = (float)(a * (k + 1) * kz);
    }
    const unsigned grid = (unsigned)((n + 255) / 256);
    const float h = (float)(dt_seconds / substeps);
    hipStream_t s = (hipStream_t)stream;
    switch (flow->nmodes) {
#define ADM1_ADVECT_CASE(M)                                                                  \
    case M:                                                                                  \
        hipLaunchKernelGGL(adm1::k_advect<M>, dim3(grid), dim3(256), 0, s, pos, ld, n, F, h, \
                           (int)substeps);                                                   \
        break;
        ADM1_ADVECT_CASE(0)
        ADM1_ADVECT_CASE(1)
        ADM1_ADVECT_CASE(2)
        ADM1_ADVECT_CASE(3)
        ADM1_ADVECT_CASE(4)
        ADM1_ADVECT_CASE(5)
        ADM1_ADVECT_CASE(6)
        ADM1_ADVECT_CASE(7)
        ADM1_ADVECT_CASE(8)
#undef ADM1_ADVECT_CASE
    default:
        return ADM1_E_OPTS;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ADM1_OK : (int)e;
}

int adm1_feed_mask(const float* pos, int64_t ld, int64_t n, double z_min, double r_max,
                   double D_zone, int32_t fidx_zone, int32_t fidx_out, double* D,
                   int32_t* fidx, uint8_t* flag, void* stream)
{
    if (!pos || !D || !fidx) return ADM1_E_NULL;
    if (n < 0 || ld < n || ld <= 0 || ld % 64 != 0) return ADM1_E_SIZE;
    if (!adm1::is_dev(pos) || !adm1::is_dev(D) || !adm1::is_dev(fidx) ||
        (flag && !adm1::is_dev(flag)))
        return ADM1_E_NOT_DEVICE;
    if (n == 0) return ADM1_OK;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(adm1::k_feed_mask, dim3(grid), dim3(256), 0, (hipStream_t)stream, pos,
                       ld, n, (float)z_min, (float)r_max, D_zone, fidx_zone, fidx_out, D, fidx,
                       flag);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ADM1_OK : (int)e;
}

}  // extern "C"
