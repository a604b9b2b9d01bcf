// HIP kernels of the per-particle ADM1 step for gfx950 (MI355X).
//
// Every particle is integrated independently over one coupling interval
// (sec. 2.3, sec. 4.3): the right-hand side of eq. 2 with the algebraic
// solves of eqs. 7-8, an adaptive Rodas4 Rosenbrock step, and the bordered
// Newton matrix of the 28 differential entries plus the two constraints.
//
// This file holds the one-lane-per-particle kernels (step with a dense
// bordered LU, the paper's fixed-step explicit scheme, right-hand side,
// Jacobian, gas flux).  The two-lanes-per-particle register-resident step
// lives in adm1_step_sparse2.hip.
#include <hip/hip_runtime.h>

#include "adm1_fixed.h"
#include "adm1_kernels.h"
#include "adm1_count.h"
#include "adm1_model.h"
#include "adm1_rodas4.h"

namespace adm1 {

constexpr int NB = 30;  // bordered system: 28 differential + eq. 7 + eq. 8 rows

// Dense LU with partial pivoting of the bordered matrix (row-major NBxNB).
__device__ static bool lu_dense(double* M, int* piv)
{
    for (int k = 0; k < NB; ++k) {
        int pr = k;
        double best = fabs(M[k * NB + k]);
        for (int i = k + 1; i < NB; ++i) {
            const double v = fabs(M[i * NB + k]);
            if (v > best) { best = v; pr = i; }
        }
        piv[k] = pr;
        if (!(best > 0.0) || !(best < INFINITY)) return false;
        if (pr != k)
            for (int j = 0; j < NB; ++j) {
                const double t = M[k * NB + j];
                M[k * NB + j] = M[pr * NB + j];
                M[pr * NB + j] = t;
            }
        const double inv = 1.0 / M[k * NB + k];
        for (int i = k + 1; i < NB; ++i) {
            const double l = M[i * NB + k] * inv;
            M[i * NB + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < NB; ++j) M[i * NB + j] -= l * M[k * NB + j];
        }
    }
    return true;
}

__device__ static void lu_dense_solve(const double* M, const int* piv, double* b)
{
    for (int k = 0; k < NB; ++k)
        if (piv[k] != k) { const double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 1; i < NB; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= M[i * NB + k] * b[k];
        b[i] = s;
    }
    for (int i = NB - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < NB; ++k) s -= M[i * NB + k] * b[k];
        b[i] = s / M[i * NB + i];
    }
}

// Bordered Newton matrix [alpha I - f_y, -f_z; g_y, g_z] (eq. 8 row negated).
__device__ static void build_dense(const DevParams& p, const Partials& d, double alpha,
                                   double D, double* M)
{
    for (int k = 0; k < NB * NB; ++k) M[k] = 0.0;
#include <adm1_jac_dense.inc>
}

__device__ __forceinline__ double rms_scaled(const DevParams& p, const double* v,
                                             const double* y)
{
    double e = 0.0;
    for (int i = 0; i < NY; ++i) {
        const double sc = p.atol[i] + p.rtol * fabs(y[i]);
        e += (v[i] / sc) * (v[i] / sc);
    }
    return sqrt(e / NY);
}

// Starting step (Hairer, Norsett & Wanner, Solving ODEs I, sec. II.4), order 4.
template <typename R>
__device__ static double initial_step(const DevParams& p, const TConst& c, const double* y0,
                                      double D, const double* sin, double dt, double H,
                                      double S, int& it)
{
    double f0[NY], y1[NY], f1[NY];
    if (rhs<R>(p, c, y0, D, sin, H, S, f0, it)) return dt;
    const double d0 = rms_scaled(p, y0, y0), d1 = rms_scaled(p, f0, y0);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > dt) h0 = dt;
    for (int i = 0; i < NY; ++i) y1[i] = y0[i] + h0 * f0[i];
    if (rhs<R>(p, c, y1, D, sin, H, S, f1, it)) return h0;
    for (int i = 0; i < NY; ++i) f1[i] -= f0[i];
    const double d2 = rms_scaled(p, f1, y0) / h0;
    const double dm = fmax(d1, d2);
    const double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : exp(0.2 * log(0.01 / dm));
    return fmin(fmin(100.0 * h0, h1), dt);
}

__device__ __forceinline__ bool all_finite(const double* v, int n)
{
    bool ok = true;
    for (int i = 0; i < n; ++i) ok = ok & isfinite(v[i]);
    return ok;
}

// Linear-algebra policies for the bordered Newton matrix of one particle.
struct LinDense {  // dense LU with partial pivoting (in scratch memory)
    double M[NB * NB];
    int piv[NB];
    __device__ bool setup(const DevParams& p, const Partials& d, double alpha, double D)
    {
        build_dense(p, d, alpha, D, M);
        return lu_dense(M, piv);
    }
    __device__ void solve(double* b) const { lu_dense_solve(M, piv, b); }
};

#include <adm1_jac_sparse1.inc>

struct LinSparse1 {  // generated static-order sparse LU, named scalars
    ADM1_SP_DECL
    __device__ bool setup(const DevParams& p, const Partials& d, double alpha, double D)
    {
        ADM1_SP_BUILD(alpha, D);
        bool ok = true;
        ADM1_SP_FACTOR(ok, p.pivot_floor, alpha);
        return ok;
    }
    __device__ void solve(double* b) const { ADM1_SP_SOLVE(b); }
};

#include <adm1_jac_sparse1_lds.inc>

// The LDS of the one-lane kernel with the matrix in LDS: ADM1_SPL_NNZ
// entries of each of the 64 particles of the workgroup (124 KB; one
// workgroup per compute unit).
__device__ __forceinline__ double* lds_lu()
{
    __shared__ double buf[ADM1_SPL_NNZ * 64];
    return buf;
}

struct LinSparse1Lds {  // generated static-order sparse LU, matrix in LDS
    double* Lm;  // this lane's entry 0; entry e at Lm[e * 64]
    ADM1_SPL_DECL
    __device__ LinSparse1Lds() : Lm(lds_lu() + threadIdx.x) {}
#define ADM1_SPL_M(e) Lm[(e) * 64]
    __device__ bool setup(const DevParams& p, const Partials& d, double alpha, double D)
    {
        ADM1_SPL_BUILD(alpha, D);
        bool ok = true;
        ADM1_SPL_FACTOR(ok, p.pivot_floor, alpha);
        return ok;
    }
    __device__ void solve(double* b) const { ADM1_SPL_SOLVE(b); }
#undef ADM1_SPL_M
};

// One coupling interval for one particle on one lane.  Inlined: a call made
// under a partial exec mask (lanes past n, lanes with invalid input) may
// overwrite what the inactive lanes keep in caller-saved registers.
template <typename R, typename Lin>
__device__ __forceinline__ static int integrate1(const DevParams& p, const TConst& c, double* y,
                                                 double D, const double* sin, double dt,
                                                 double& H, double& Sh2, double& hlast, int* cnt)
{
    Lin lin;
    double u[kR4Stages][NY];
    double arg[NY], f[NY], b[NB];
    int it = 0;
    {
        double Ht = H, St = Sh2;
        if (rhs<R>(p, c, y, D, sin, Ht, St, f, it)) { cnt[2] = it; return 1; }
        H = Ht;
        Sh2 = St;
    }
    double h = hlast > 0.0 ? fmin(dt, hlast) : initial_step<R>(p, c, y, D, sin, dt, H, Sh2, it);
    const double hmin = 1e-14 * dt;
    double t = 0.0;
    bool reject_prev = false;
    int n = 0, st = 0;
    for (;;) {
        if (n >= p.max_steps) { st = 3; break; }
        if (h < hmin) { st = 2; break; }
        double hs = h;
        bool clip = false;
        if (t + 1.01 * hs >= dt) { hs = dt - t; clip = true; }
        double err = INFINITY;
        bool ok = true;
        // stage 1 right-hand side and the algebraic roots at y0
        ok = rhs<R>(p, c, y, D, sin, H, Sh2, f, it) == 0;
        if (ok) {
            Partials d;
            partials(p, c, y, H, Sh2, d);
            ok = lin.setup(p, d, 1.0 / (kR4Gamma * hs), D);
        }
        for (int s = 0; ok && s < kR4Stages; ++s) {
            if (s > 0) {
                for (int i = 0; i < NY; ++i) {
                    double a = y[i];
                    for (int j = 0; j < s; ++j) a += kR4A[s][j] * u[j][i];
                    arg[i] = a;
                }
                ok = rhs<R>(p, c, arg, D, sin, H, Sh2, f, it) == 0;
                if (!ok) break;
            } else {
                for (int i = 0; i < NY; ++i) arg[i] = y[i];
            }
            const double ih = 1.0 / hs;
            for (int i = 0; i < NY; ++i) {
                double v = f[i];
                for (int j = 0; j < s; ++j) v += kR4C[s][j] * ih * u[j][i];
                b[i] = v;
            }
            b[NY] = 0.0;
            b[NY + 1] = 0.0;
            lin.solve(b);
            for (int i = 0; i < NY; ++i) u[s][i] = b[i];
        }
        double y1[NY];
        if (ok) {
            double e = 0.0;
            for (int i = 0; i < NY; ++i) {
                y1[i] = arg[i] + u[5][i];
                const double sc = p.atol[i] + p.rtol * fmax(fabs(y[i]), fabs(y1[i]));
                e += (u[5][i] / sc) * (u[5][i] / sc);
            }
            err = sqrt(e / NY);
            ok = all_finite(y1, NY) & isfinite(err);
        }
        ++n;
        const double fac = ok ? step_factor(err) : 0.2;
        double hnew = hs * fac;
        if (ok && err <= 1.0) {
            ++cnt[0];
            for (int i = 0; i < NY; ++i) y[i] = y1[i];
            if (reject_prev && hnew > hs) hnew = hs;
            reject_prev = false;
            if (clip) {
                hlast = fmax(hnew, h);
                break;
            }
            t += hs;
            h = hnew;
        } else {
            ++cnt[1];
            reject_prev = true;
            h = hnew;
        }
    }
    if (st == 0) {
        // algebraic write-back at the end of the interval
        if (rhs<R>(p, c, y, D, sin, H, Sh2, f, it)) st = 1;
    }
    cnt[2] = it;
    return st;
}

// Writes the 35-entry state of a particle from y and the algebraic roots.
__device__ __forceinline__ void store_state(const DevParams& p, const TConst& c,
                                            double* state, int64_t ld, int64_t i,
                                            const double* y, double H, double Sh2)
{
    for (int k = 0; k < NY; ++k) state[state_row(k) * ld + i] = y[k];
    state[ROW_SH2 * ld + i] = Sh2;
    state[26 * ld + i] = p.K_a_va * y[Sva] / (p.K_a_va + H);
    state[27 * ld + i] = p.K_a_bu * y[Sbu] / (p.K_a_bu + H);
    state[28 * ld + i] = p.K_a_pro * y[Spro] / (p.K_a_pro + H);
    state[29 * ld + i] = p.K_a_ac * y[Sac] / (p.K_a_ac + H);
    state[30 * ld + i] = c.K_a_co2 * y[SIC] / (c.K_a_co2 + H);
    state[31 * ld + i] = c.K_a_IN * y[SIN] / (c.K_a_IN + H);
}

template <typename R, typename Lin>
__global__ void __launch_bounds__(64, 1) k_step1(StepArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const DevParams& p = a.p;
    double y[NY];
    for (int k = 0; k < NY; ++k) y[k] = a.state[state_row(k) * a.ld + i];
    const double T = a.T[i], D = a.D[i];
    const int fi = a.fidx[i];
    double H = a.H ? a.H[i] : -1.0, hl = a.hlast ? a.hlast[i] : -1.0;
    double Sh2 = a.state[ROW_SH2 * a.ld + i];
    int cnt[3] = {0, 0, 0};
    int st;
    if (!all_finite(y, NY) || !isfinite(T) || !isfinite(D) || !(T > 0.0) || fi < 0 ||
        fi >= a.n_feed) {
        st = 4;
    } else {
        const double* sin = a.S_in + (int64_t)fi * NLIQ;
        bool fin = true;
        for (int k = 0; k < NLIQ; ++k) fin = fin & isfinite(sin[k]);
        if (!fin) {
            st = 4;
        } else {
            TConst c = tconst(p, T);
            c.arr *= phase_factor(a.phase, a.phase_kin, i);
            st = integrate1<R, Lin>(p, c, y, D, sin, a.dt, H, Sh2, hl, cnt);
            if (st == 0) {
                store_state(p, c, a.state, a.ld, i, y, H, Sh2);
                if (a.H) a.H[i] = H;
                if (a.hlast) a.hlast[i] = hl;
                for (int k = 0; k < NY; ++k)
                    if (y[k] < 0.0) st |= 0x80;
            }
        }
    }
    a.status[i] = (uint8_t)st;
    if (a.nsteps) {
        a.nsteps[i] = cnt[0];
        a.nsteps[a.ld + i] = cnt[1];
        a.nsteps[2 * a.ld + i] = cnt[2];
    }
}

// The paper's fixed-step scheme: `substeps` equal explicit steps over the
// interval, explicit Euler (M = 0) or classical RK4 (M = 1), every
// right-hand-side evaluation solving eqs. 7-8 at the current differential
// state (warm-started from the previous roots); then the algebraic
// write-back.  Status: 0 ok, 1 an algebraic solve failed, 2 a step produced a
// non-finite state, 4 non-finite or invalid input; bit 0x80 flags a negative
// differential entry.  A failed particle keeps its input.
template <typename R, int M>
__device__ __forceinline__ void fixed_body(const FixedArgs& a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const DevParams& p = a.p;
    double y[NY];
    for (int k = 0; k < NY; ++k) y[k] = a.state[state_row(k) * a.ld + i];
    const double T = a.T[i], D = a.D[i];
    const int fi = a.fidx[i];
    double H = a.H ? a.H[i] : -1.0;
    double Sh2 = a.state[ROW_SH2 * a.ld + i];
    int it = 0, st = 0;
    const double* sin = nullptr;
    if (!all_finite(y, NY) || !isfinite(T) || !isfinite(D) || !(T > 0.0) || fi < 0 ||
        fi >= a.n_feed) {
        st = 4;
    } else {
        sin = a.S_in + (int64_t)fi * NLIQ;
        for (int k = 0; k < NLIQ; ++k)
            if (!isfinite(sin[k])) st = 4;
    }
    if (st == 0) {
        TConst c = tconst(p, T);
        c.arr *= phase_factor(a.phase, a.phase_kin, i);
        const double h = a.dt / a.substeps;
        double f[NY];
        for (int s = 0; s < a.substeps && st == 0; ++s) {
            // Euler re-reads the feed row every substep (an empty asm hides
            // the pointer) instead of holding 26 inflows in registers
            // throughout; RK4, at one wave per SIMD anyway, keeps them
            const double* sinv = sin;
            if (M == 0) asm volatile("" : "+v"(sinv));
            if (M == 0) {
                // Euler update written in place: rhs_in reads every entry for
                // the last time in the expression of its own derivative, so
                // y[k] may take its new value as soon as f_k is formed
                if (rhs_in<R>(p, c, y, D, FeedInflow{D, sinv}, H, Sh2,
                              [&y, h](int k, double v) { y[k] = fma(h, v, y[k]); }, it)) {
                    st = 1;
                    break;
                }
            } else {
                double y0[NY], acc[NY];
                for (int k = 0; k < NY; ++k) y0[k] = y[k];
                // stages 1-3: f at the stage argument, then the next argument
                const double wt[3] = {1.0, 2.0, 2.0};
                const double ah[3] = {0.5 * h, 0.5 * h, h};
                for (int q = 0; q < 3 && st == 0; ++q) {
                    if (rhs<R>(p, c, y, D, sinv, H, Sh2, f, it)) {
                        st = 1;
                        break;
                    }
                    for (int k = 0; k < NY; ++k) {
                        acc[k] = q ? fma(wt[q], f[k], acc[k]) : f[k];
                        y[k] = fma(ah[q], f[k], y0[k]);
                    }
                }
                if (st) break;
                if (rhs<R>(p, c, y, D, sinv, H, Sh2, f, it)) {
                    st = 1;
                    break;
                }
                for (int k = 0; k < NY; ++k) y[k] = fma(h / 6.0, acc[k] + f[k], y0[k]);
            }
            if (!all_finite(y, NY)) st = 2;
        }
        // algebraic write-back: S_H+ and S_h2 at the final differential state
        if (st == 0 &&
            rhs_in<R>(p, c, y, D, FeedInflow{D, sin}, H, Sh2, [](int, double) {}, it, true))
            st = 1;
        if (st == 0) {
            store_state(p, c, a.state, a.ld, i, y, H, Sh2);
            if (a.H) a.H[i] = H;
            for (int k = 0; k < NY; ++k)
                if (y[k] < 0.0) st |= 0x80;
        }
    }
    a.status[i] = (uint8_t)st;
    if (a.newton) a.newton[i] = it;
}

// Euler fits two waves per SIMD (its state is updated in place); RK4 keeps
// four stage vectors and runs at one wave per SIMD without spills.
template <typename R>
__global__ void __launch_bounds__(64, 2) k_fixed_euler(FixedArgs a)
{
    fixed_body<R, 0>(a);
}

template <typename R>
__global__ void __launch_bounds__(64) k_fixed_rk4(FixedArgs a)
{
    fixed_body<R, 1>(a);
}

template <typename R>
__global__ void __launch_bounds__(64) k_rhs(RhsArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const DevParams& p = a.p;
    double y[NY], f[NY];
    for (int k = 0; k < NY; ++k) y[k] = a.state[state_row(k) * a.ld + i];
    TConst c = tconst(p, a.T[i]);
    c.arr *= phase_factor(a.phase, a.phase_kin, i);
    const int fi = a.fidx[i];
    if (fi < 0 || fi >= a.n_feed) {
        for (int k = 0; k < NY; ++k) a.dxdt[k * a.ld_out + i] = NAN;
        if (a.H_out) a.H_out[i] = NAN;
        if (a.status) a.status[i] = 4;
        return;
    }
    const double* sin = a.S_in + (int64_t)fi * NLIQ;
    double H = -1.0, S = a.state[ROW_SH2 * a.ld + i];
    int it = 0;
    const int rc = rhs<R>(p, c, y, a.D[i], sin, H, S, f, it);
    for (int k = 0; k < NY; ++k) a.dxdt[k * a.ld_out + i] = rc ? NAN : f[k];
    if (a.H_out) a.H_out[i] = rc ? NAN : H;
    if (a.status) a.status[i] = rc ? 1 : 0;
}

// Eq. 7 alone: S_H+ of each particle's totals (the ions as equilibrium
// fractions), by the same Newton iteration the right-hand side uses.
__global__ void __launch_bounds__(64) k_solve_ph(PhArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const DevParams& p = a.p;
    double y[NY];
    bool fin = true;
    for (int k = 0; k < NY; ++k) {
        y[k] = a.state[state_row(k) * a.ld + i];
        fin = fin & isfinite(y[k]);
    }
    const double T = a.T[i];
    fin = fin & isfinite(T) & (T > 0.0);
    double H = a.guess ? a.guess[i] : -1.0;
    int it = 0;
    int st = 4;
    if (fin) {
        const TConst c = tconst(p, T);
        st = solve_H(p, c, y, H, it) ? 1 : 0;
    }
    a.H_out[i] = st ? NAN : H;
    if (a.pH_out) a.pH_out[i] = st ? NAN : -log10(H);
    if (a.status) a.status[i] = (uint8_t)st;
}

// Outcome counters: one pass over the status bytes by a fixed grid of
// kCountBlocks blocks, block sums in LDS, each block's sums stored to its own
// row of the partials (the host adds the rows).  A thread takes 16
// consecutive bytes per pass as 16 independent loads, so each wave keeps
// 1 KB in flight; the ragged end is read byte by byte.
__device__ __forceinline__ void tally_status(unsigned v, unsigned int (&loc)[kFailSlots])
{
    const unsigned code = v & 0x7Fu;
    loc[0] += code != 0;
    loc[1] += code == 1;
    loc[2] += code == 2;
    loc[3] += code == 3;
    loc[4] += code == 4;
    loc[5] += (code == 0) & ((v & 0x80u) != 0);
    loc[6] += 1;
}

__global__ void __launch_bounds__(256) k_count_status(const uint8_t* status, int64_t n,
                                                      unsigned long long* part_out)
{
    __shared__ unsigned int part[kFailSlots][256];
    unsigned int loc[kFailSlots] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 16;
    for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; i0 < n;
         i0 += stride) {
        if (i0 + 16 <= n) {
            unsigned v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = status[i0 + j];
#pragma unroll
            for (int j = 0; j < 16; ++j) tally_status(v[j], loc);
        } else {
            for (int64_t i = i0; i < n; ++i) tally_status(status[i], loc);
        }
    }
    for (int k = 0; k < kFailSlots; ++k) part[k][threadIdx.x] = loc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < kFailSlots; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + w];
        __syncthreads();
    }
    // every block writes all its slots on every call: no reset, no atomics
    if (threadIdx.x < kFailSlots)
        part_out[blockIdx.x * kFailSlots + threadIdx.x] = part[threadIdx.x][0];
}

// Total Jacobian: minus the Schur complement of the constraint block of the
// bordered matrix taken at alpha = 0.
__global__ void __launch_bounds__(64) k_jacobian(RhsArgs a, double* J)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const DevParams& p = a.p;
    double y[NY], f[NY], M[NB * NB];
    for (int k = 0; k < NY; ++k) y[k] = a.state[state_row(k) * a.ld + i];
    TConst c = tconst(p, a.T[i]);
    c.arr *= phase_factor(a.phase, a.phase_kin, i);
    double* Jo = J + i * NY * NY;
    const int fi = a.fidx[i];
    if (fi < 0 || fi >= a.n_feed) {
        for (int k = 0; k < NY * NY; ++k) Jo[k] = NAN;
        if (a.status) a.status[i] = 4;
        return;
    }
    const double* sin = a.S_in + (int64_t)fi * NLIQ;
    double H = -1.0, S = a.state[ROW_SH2 * a.ld + i];
    int it = 0;
    const double D = a.D[i];
    const int rc = rhs<double>(p, c, y, D, sin, H, S, f, it);
    if (a.status) a.status[i] = rc ? 1 : 0;
    if (rc) {
        for (int k = 0; k < NY * NY; ++k) Jo[k] = NAN;
        return;
    }
    Partials d;
    partials(p, c, y, H, S, d);
    build_dense(p, d, 0.0, D, M);
    const double g00 = M[28 * NB + 28], g01 = M[28 * NB + 29];
    const double g10 = M[29 * NB + 28], g11 = M[29 * NB + 29];
    const double det = g00 * g11 - g01 * g10;
    const double i00 = g11 / det, i01 = -g01 / det, i10 = -g10 / det, i11 = g00 / det;
    for (int r = 0; r < NY; ++r) {
        const double b0 = M[r * NB + 28], b1 = M[r * NB + 29];
        const double w0 = b0 * i00 + b1 * i10, w1 = b0 * i01 + b1 * i11;
        for (int k = 0; k < NY; ++k)
            Jo[r * NY + k] = -M[r * NB + k] + w0 * M[28 * NB + k] + w1 * M[29 * NB + k];
    }
}

// Gas flows per particle and per-block partial totals (fixed order).
__global__ void __launch_bounds__(256) k_gasflux(GasArgs a)
{
    __shared__ double red[4][256];
    const DevParams& p = a.p;
    const int64_t begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = begin + a.chunk < a.n ? begin + a.chunk : a.n;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = begin + threadIdx.x; i < end; i += 256) {
        const double T = a.T[i];
        const double RT = p.R * T;
        const double vh = p.inv_T_base - 1.0 / T;
        const double p_h2o = p.p_h2o_base * exp(p.p_h2o_coef * vh);
        const double ph2 = a.state[32 * a.ld + i] * RT * (1.0 / 16.0);
        const double pch4 = a.state[33 * a.ld + i] * RT * (1.0 / 64.0);
        const double pco2 = a.state[34 * a.ld + i] * RT;
        const double P = ph2 + pch4 + pco2 + p_h2o;
        const double V = a.V_liq ? a.V_liq[i] : 1.0;
        const double q = P > p.P_atm ? V * p.kp * (P - p.P_atm) * P / p.P_atm : 0.0;
        const double iP = 1.0 / P;
        if (a.q_gas) a.q_gas[i] = q;
        if (a.q_ch4) a.q_ch4[i] = q * pch4 * iP;
        acc[0] += q;
        acc[1] += q * ph2 * iP;
        acc[2] += q * pch4 * iP;
        acc[3] += q * pco2 * iP;
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) a.partial[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_gasflux_final(const double* partial, int nblocks,
                                                       double* totals)
{
    __shared__ double red[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int k = 0; k < 4; ++k) acc[k] += partial[b * 4 + k];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) totals[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Launchers (host)
// ---------------------------------------------------------------------------
hipError_t launch_step1(const StepArgs& a, int rate_precision, int lin, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) return hipSuccess;
    const bool f32 = rate_precision != 0;
    if (lin == 1) {
        if (f32) hipLaunchKernelGGL((k_step1<float, LinSparse1>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_step1<double, LinSparse1>), dim3(grid), dim3(64), 0, s, a);
    } else if (lin == 2) {
        if (f32)
            hipLaunchKernelGGL((k_step1<float, LinSparse1Lds>), dim3(grid), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL((k_step1<double, LinSparse1Lds>), dim3(grid), dim3(64), 0, s, a);
    } else {
        if (f32) hipLaunchKernelGGL((k_step1<float, LinDense>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_step1<double, LinDense>), dim3(grid), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_fixed(const FixedArgs& a, int rate_precision, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) return hipSuccess;
    if (a.method == 0) {
        if (rate_precision)
            hipLaunchKernelGGL(k_fixed_euler<float>, dim3(grid), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL(k_fixed_euler<double>, dim3(grid), dim3(64), 0, s, a);
    } else {
        if (rate_precision)
            hipLaunchKernelGGL(k_fixed_rk4<float>, dim3(grid), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL(k_fixed_rk4<double>, dim3(grid), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_rhs(const RhsArgs& a, int rate_precision, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) return hipSuccess;
    if (rate_precision)
        hipLaunchKernelGGL(k_rhs<float>, dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(k_rhs<double>, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_solve_ph(const PhArgs& a, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve_ph, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_count_status(const uint8_t* status, int64_t n, unsigned long long* counts,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_count_status, dim3(kCountBlocks), dim3(256), 0, s, status,
                       n > 0 ? n : 0, counts);
    return hipGetLastError();
}

hipError_t launch_jacobian(const RhsArgs& a, double* J, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobian, dim3(grid), dim3(64), 0, s, a, J);
    return hipGetLastError();
}

hipError_t launch_gasflux(const GasArgs& a, int nblocks, double* totals, hipStream_t s)
{
    hipLaunchKernelGGL(k_gasflux, dim3(nblocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gasflux_final, dim3(1), dim3(256), 0, s, a.partial, nblocks, totals);
    return hipGetLastError();
}

}  // namespace adm1
