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
// stored as FP32 structure-of-arrays pos[3][ld] (x, y, z in m) but advanced
// in FP64 over all substeps of a call.  The meridional part (u_r, u_z) is
// axisymmetric and so commutes with the rotation: each substep is a
// classical RK4 step of the meridional flow followed by the turn of the
// (x, y) plane by Omega h (RK4 on the rotation itself would shrink every
// orbit by about 2 % per 1 s substep at 12 rpm).  The turn is three shears,
// x -= t y, y += s x, x -= t y with t = tan(Omega h / 2), s = sin(Omega h):
// each shear has determinant 1 whatever the rounding of t and s, so orbits
// stay closed.  A particle that still crosses a wall or the lid by rounding
// is reflected back inside: the boundary is an invariant set of the flow, so
// a particle placed on it would stay there for good.
//
// Why FP64: the axis is invariant too, and where the meridional flow
// converges radially onto it (an axial stagnation point z1 with u_z ~
// c (z - z1), c > 0) a particle on the converging side leaves along the axis
// only as fast as |z - z1| grows.  In FP32 that growth per substep falls
// below half an ulp of z within a few tenths of a micrometre of z1 (and the
// FP32 velocity carries rounding noise of that order), so z stops moving
// while r keeps shrinking geometrically down to denormals; such particles
// then collect at the next stagnation point on the axis, dozens at one
// position after a few hour-long intervals, where the exact flow (which
// conserves r^2 (z - z1)) keeps them apart.  In FP64 the band of lost
// increments is ~1e-17 m wide and no particle falls into it.  The price is
// the FP64 issue rate (half the FP32 vector rate); one FP64 sine and cosine
// per substep, the RK4 stages turning that angle by their short offsets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "adm1.h"

namespace adm1 {
namespace {

struct Field {
    double tan_half, sin_wh;  // turn of one substep as three shears
    double R, H;
    double kz;  // pi / H
    // per mode k (1-based): a_k (axial) and a_k k pi / H (radial), so the
    // velocity is u_r/r = -(R^2 - r^2) sum_k rad_k cos(k kz z),
    // u_z = (2 R^2 - 4 r^2) sum_k ax_k sin(k kz z)
    double ax[ADM1_FLOW_MODES];
    double rad[ADM1_FLOW_MODES];
};

// Meridional velocity (the rotation is applied exactly, outside RK4) of NM
// modes at sin and cos of kz z given, as u_r / r and u_z.  sin and cos of
// k kz z come from those of kz z by angle addition.
template <int NM>
__device__ __forceinline__ void velocity(const Field& F, double x, double y, double s1, double c1,
                                         double& g, double& uz)
{
    const double r2 = x * x + y * y;
    const double R2 = F.R * F.R;
    double s = s1, c = c1, sc = 0.0, ss = 0.0;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        sc = fma(F.rad[k], c, sc);
        ss = fma(F.ax[k], s, ss);
        const double sn = fma(s, c1, c * s1);
        c = fma(c, c1, -s * s1);
        s = sn;
    }
    g = -(R2 - r2) * sc;
    uz = (2.0 * R2 - 4.0 * r2) * ss;
}

// sin and cos of (theta + e) from those of theta.  An RK4 stage sits a short
// way from the substep's start (|e| = kz |dz| is ~0.1 rad at the field's
// speeds), so sin e and cos e come from their Taylor series through e^11 and
// e^12 (truncation below 1e-17 for |e| <= 0.25); longer offsets take the
// library sine and cosine.
__device__ __forceinline__ void turn_angle(double sb, double cb, double e, double& s, double& c)
{
    double se, ce;
    if (fabs(e) <= 0.25) {
        const double e2 = e * e;
        double p = -1.0 / 39916800.0;
        p = fma(p, e2, 1.0 / 362880.0);
        p = fma(p, e2, -1.0 / 5040.0);
        p = fma(p, e2, 1.0 / 120.0);
        p = fma(p, e2, -1.0 / 6.0);
        se = fma(e * e2, p, e);
        double q = 1.0 / 479001600.0;
        q = fma(q, e2, -1.0 / 3628800.0);
        q = fma(q, e2, 1.0 / 40320.0);
        q = fma(q, e2, -1.0 / 720.0);
        q = fma(q, e2, 1.0 / 24.0);
        q = fma(q, e2, -0.5);
        ce = fma(e2, q, 1.0);
    } else {
        sincos(e, &se, &ce);
    }
    s = fma(sb, ce, cb * se);
    c = fma(cb, ce, -sb * se);
}

// Reflect a particle that crossed the wall, the bottom or the lid back into
// the tank (then clamp, for overshoots larger than the tank).
__device__ __forceinline__ void reflect_tank(const Field& F, double& x, double& y, double& z)
{
    const double r2 = x * x + y * y;
    if (r2 > F.R * F.R) {
        const double r = sqrt(r2);
        const double f = fmax(2.0 * F.R - r, 0.0) / r;
        x *= f;
        y *= f;
    }
    if (z < 0.0) z = -z;
    if (z > F.H) z = 2.0 * F.H - z;
    z = fmin(fmax(z, 0.0), F.H);
}

template <int NM>
__global__ void __launch_bounds__(256) k_advect(float* pos, int64_t ld, int64_t n, Field F,
                                                double h, int nsub)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = pos[i], y = pos[ld + i], z = pos[2 * ld + i];
    const double hh = 0.5 * h, h6 = h / 6.0;
    for (int s = 0; s < nsub; ++s) {
        // u_x = g x and u_y = g y: every stage scales x and y alike
        double g1, g2, g3, g4, w1, w2, w3, w4, sb = 0.0, cb = 1.0, st = 0.0, ct = 1.0;
        if (NM > 0) sincos(F.kz * z, &sb, &cb);
        velocity<NM>(F, x, y, sb, cb, g1, w1);
        const double m2 = fma(hh, g1, 1.0);
        if (NM > 0) turn_angle(sb, cb, F.kz * (hh * w1), st, ct);
        velocity<NM>(F, m2 * x, m2 * y, st, ct, g2, w2);
        const double m3 = fma(hh * g2, m2, 1.0);
        if (NM > 0) turn_angle(sb, cb, F.kz * (hh * w2), st, ct);
        velocity<NM>(F, m3 * x, m3 * y, st, ct, g3, w3);
        const double m4 = fma(h * g3, m3, 1.0);
        if (NM > 0) turn_angle(sb, cb, F.kz * (h * w3), st, ct);
        velocity<NM>(F, m4 * x, m4 * y, st, ct, g4, w4);
        const double m = fma(h6, g1 + 2.0 * g2 * m2 + 2.0 * g3 * m3 + g4 * m4, 1.0);
        x *= m;
        y *= m;
        z = fma(h6, w1 + 2.0 * w2 + 2.0 * w3 + w4, z);
        x = fma(-F.tan_half, y, x);
        y = fma(F.sin_wh, x, y);
        x = fma(-F.tan_half, y, x);
        reflect_tank(F, x, y, z);
    }
    pos[i] = (float)x;
    pos[ld + i] = (float)y;
    pos[2 * ld + i] = (float)z;
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
    F.tan_half = std::tan(0.5 * wh);
    F.sin_wh = std::sin(wh);
    F.R = flow->R;
    F.H = flow->H;
    const double kz = 3.14159265358979323846 / flow->H;
    F.kz = kz;
    for (int k = 0; k < ADM1_FLOW_MODES; ++k) {
        const double a = k < flow->nmodes ? flow->a[k] : 0.0;
        F.ax[k] = a;
        F.rad[k] = a * (k + 1) * kz;
    }
    const unsigned grid = (unsigned)((n + 255) / 256);
    const double h = dt_seconds / substeps;
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
