// ADM1 reaction model for one particle: device functions shared by the
// step, right-hand-side and gate kernels.
//
// A particle is a CSTR (sec. 2.3) obeying the mass balance of eq. 2 with the
// standard ADM1 kinetics (sec. 2.2), the inhibition forms of eqs. 3-6, the
// charge balance of eq. 7 (solved for S_H+) and the hydrogen balance of
// eq. 8 (solved for S_h2).  The 28 differential entries y are integrated;
// S_H+ and S_h2 are algebraic and re-solved at every evaluation.
//
// Integration order of y (indices below) and the 35-entry state rows:
//   y  0..6  S_su S_aa S_fa S_va S_bu S_pro S_ac   rows 0..6
//   y  7..10 S_ch4 S_IC S_IN S_I                   rows 8..11
//   y 11..22 X_xc X_ch X_pr X_li X_su..X_h2 X_I    rows 12..23
//   y 23..24 S_cat S_an                            rows 24..25
//   y 25..27 G_h2 G_ch4 G_co2                      rows 32..34
// Algebraic rows: 7 S_h2, 26..31 S_va-, S_bu-, S_pro-, S_ac-, S_hco3-, S_nh3.
#pragma once
#include <hip/hip_runtime.h>

#include "adm1_devparams.h"

namespace adm1 {

enum YIdx {
    Ssu, Saa, Sfa, Sva, Sbu, Spro, Sac, Sch4, SIC, SIN, SI, Xxc, Xch, Xpr, Xli, Xsu, Xaa,
    Xfa, Xc4, Xpro, Xac, Xh2, XI, Scat, San, Gh2, Gch4, Gco2, NY
};
constexpr int NX = 35;
constexpr int NLIQ = 26;
constexpr int ROW_SH2 = 7;

__host__ __device__ constexpr int state_row(int k)
{
    return k < 7 ? k : (k < 25 ? k + 1 : k + 7);
}

#include <adm1_partials.inc>
#include <adm1_stoich.inc>

// Reciprocal of a finite non-zero x: the hardware estimate refined by two
// Newton-Raphson steps (the error squares at each step, so the estimate's
// error falls far below the FP64 rounding).
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float frcp(float x) { return 1.0f / x; }

struct TConst {
    double RT, K_w, K_a_co2, K_a_IN, K_H_h2, K_H_ch4, K_H_co2, p_h2o, arr;
};

// Van't Hoff constants and the Arrhenius factor at temperature T (K).
__device__ __forceinline__ TConst tconst(const DevParams& p, double T)
{
    TConst c;
    const double vh = p.inv_T_base - 1.0 / T;
    c.RT = p.R * T;
    c.K_w = p.K_w_base * exp(p.dH_w_R100 * vh);
    c.K_a_co2 = p.K_a_co2_base * exp(p.dH_a_co2_R100 * vh);
    c.K_a_IN = p.K_a_IN_base * exp(p.dH_a_IN_R100 * vh);
    c.K_H_h2 = p.K_H_h2_base * exp(p.dH_H_h2_R100 * vh);
    c.K_H_ch4 = p.K_H_ch4_base * exp(p.dH_H_ch4_R100 * vh);
    c.K_H_co2 = p.K_H_co2_base * exp(p.dH_H_co2_R100 * vh);
    c.p_h2o = p.p_h2o_base * exp(p.p_h2o_coef * vh);
    c.arr = exp(p.Ea_R100 * (p.inv_T_ref_kin - 1.0 / T));
    return c;
}

// The kinetic factor of particle i's phase (sec. 5, several particle kinds):
// it scales every biochemical rate, and every rate carries the Arrhenius
// factor, so callers multiply TConst::arr by it.  No phase array: factor 1.
__device__ __forceinline__ double phase_factor(const uint8_t* phase, const double* kin,
                                               int64_t i)
{
    return phase ? kin[phase[i]] : 1.0;
}

// ---------------------------------------------------------------------------
// Eq. 7: charge balance E(S_H+) and dE/dS_H+.  The ions are the equilibrium
// fractions K/(K + S_H+) of their totals.
// ---------------------------------------------------------------------------
template <typename Y>
__device__ __forceinline__ double charge_balance(const DevParams& p, const TConst& c,
                                                 const Y& y, double H, double& dE)
{
    const double iIN = frcp(c.K_a_IN + H), iCO2 = frcp(c.K_a_co2 + H);
    const double iac = frcp(p.K_a_ac + H), ipro = frcp(p.K_a_pro + H);
    const double ibu = frcp(p.K_a_bu + H), iva = frcp(p.K_a_va + H);
    const double iH = frcp(H);
    const double nh3 = c.K_a_IN * y[SIN] * iIN;
    const double hco3 = c.K_a_co2 * y[SIC] * iCO2;
    const double ac = p.K_a_ac * y[Sac] * iac * (1.0 / 64.0);
    const double pro = p.K_a_pro * y[Spro] * ipro * (1.0 / 112.0);
    const double bu = p.K_a_bu * y[Sbu] * ibu * (1.0 / 160.0);
    const double va = p.K_a_va * y[Sva] * iva * (1.0 / 208.0);
    const double kw = c.K_w * iH;
    dE = 1.0 + nh3 * iIN + hco3 * iCO2 + ac * iac + pro * ipro + bu * ibu + va * iva +
         kw * iH;
    return y[Scat] + (y[SIN] - nh3) + H - hco3 - ac - pro - bu - va - kw - y[San];
}

// Newton on eq. 7 from the warm start H.  E is increasing and concave in S_H+
// for non-negative totals, so iterates left of the root climb monotonically
// onto it; a step from the right may overshoot left, and steps are clamped
// to a factor 10 either way to stay positive.  Returns 0 on convergence.
template <typename Y>
__device__ __forceinline__ int solve_H(const DevParams& p, const TConst& c, const Y& y,
                                       double& H, int& iters)
{
    double h = (H > 0.0 && H < 1e3) ? H : 1e-7;
    for (int it = 0; it < p.newton_maxit; ++it) {
        double dE;
        const double E = charge_balance(p, c, y, h, dE);
        if (!isfinite(E) || !isfinite(dE)) return 1;
        double hn = h - E * frcp(dE);
        if (!(hn >= 0.1 * h)) hn = 0.1 * h;
        else if (hn > 10.0 * h) hn = 10.0 * h;
        ++iters;
        const bool done = fabs(hn - h) <= p.newton_qtol * hn;
        h = hn;
        if (done) {
            H = h;
            return 0;
        }
    }
    return 1;
}

// ---------------------------------------------------------------------------
// Eq. 8: hydrogen balance.  With the S_h2-free rate factors precomputed,
//   E(S) = base + c7 I_fa(S) + c8 I_c4(S) + c10 I_pro(S) - c12 S/(K_S_h2 + S)
//          - (D + kLa) S + kLa kh
// (I_x = K_I,x / (K_I,x + S), eq. 5).  E is decreasing and convex, so Newton
// iterates left of the root climb onto it monotonically; steps below the
// domain bound -Kmin/2 are bisected towards it.
// ---------------------------------------------------------------------------
struct H2Terms {
    double base, c7, c8, c10, c12, kh;
};

__device__ __forceinline__ double h2_balance(const DevParams& p, const H2Terms& t, double D,
                                             double S, double& dE)
{
    const double ifa = frcp(p.K_I_h2_fa + S), ic4 = frcp(p.K_I_h2_c4 + S);
    const double ipro = frcp(p.K_I_h2_pro + S), ih2 = frcp(p.K_S_h2 + S);
    const double a7 = t.c7 * p.K_I_h2_fa * ifa, a8 = t.c8 * p.K_I_h2_c4 * ic4;
    const double a10 = t.c10 * p.K_I_h2_pro * ipro;
    dE = -(D + p.kLa) - a7 * ifa - a8 * ic4 - a10 * ipro - t.c12 * p.K_S_h2 * ih2 * ih2;
    return t.base + a7 + a8 + a10 - t.c12 * S * ih2 - (D + p.kLa) * S + p.kLa * t.kh;
}

__device__ __forceinline__ int solve_Sh2(const DevParams& p, const H2Terms& t, double D,
                                         double& S, int& iters)
{
    const double lo =
        -0.5 * fmin(fmin(p.K_S_h2, p.K_I_h2_fa), fmin(p.K_I_h2_c4, p.K_I_h2_pro));
    double s = (S > lo && S < 1e3) ? S : 0.0;
    for (int it = 0; it < p.newton_maxit; ++it) {
        double dE;
        const double E = h2_balance(p, t, D, s, dE);
        if (!isfinite(E) || !isfinite(dE)) return 1;
        double sn = s - E * frcp(dE);
        if (!(sn > lo)) sn = 0.5 * (s + lo);
        ++iters;
        const bool done = fabs(sn - s) <= p.newton_qtol * fabs(sn) + 1e-30;
        s = sn;
        if (done) {
            S = s;
            return 0;
        }
    }
    return 1;
}

// pH inhibition, eqs. 3-4 written in S_H+: 1 / (1 + (S_H+/K)^n).
template <typename R>
__device__ __forceinline__ R inhib_pH(R H, double invK, double n, int nint)
{
    const R r = H * (R)invK;
    R rn;
    // integer exponents 1..4 only (adm1_init refuses others): no call to a
    // power routine, which would run under a partial exec mask here
    if (nint == 1) rn = r;
    else if (nint == 2) rn = r * r;
    else if (nint == 3) rn = r * r * r;
    else { const R r2 = r * r; rn = r2 * r2; }
    return frcp((R)1 + rn);
}

// ---------------------------------------------------------------------------
// Right-hand side f(y) of the 28 differential entries.  R is the precision of
// the rates and the assembly (double, or float for the reduced-precision
// experiment); the eq. 7 and eq. 8 solves always run in FP64.
// H and Sh2 carry the warm starts in and the roots out.  Returns 0, or 1
// when an algebraic solve fails.
// ---------------------------------------------------------------------------
// Inflow term D S_in of state row k, read from the feed table.
struct FeedInflow {
    double D;
    const double* sin;
    __device__ __forceinline__ double operator()(int k) const { return D * sin[k]; }
};

template <typename R>
__device__ __forceinline__ int rhs(const DevParams& p, const TConst& c, const double* y,
                                   double D, const double* sin, double& H, double& Sh2,
                                   double* f, int& iters);

// Right-hand side with the inflow terms D S_in supplied by `inflow` (one
// accessor per storage layout of the feed).  With alg_only the evaluation
// stops once S_H+ and S_h2 are solved (nothing is written to `out`).
template <typename R, typename Y, typename Inflow, typename Out>
__device__ __forceinline__ int rhs_in(const DevParams& p, const TConst& c, const Y& y,
                                      double D, const Inflow& inflow, double& H, double& Sh2,
                                      const Out& out, int& iters, bool alg_only = false)
{
    if (solve_H(p, c, y, H, iters)) return 1;
    const R a = (R)c.arr;
    const R Hr = (R)H;
    const R I_aa = inhib_pH<R>(Hr, p.pH_invK[0], p.pH_n[0], p.pH_nint[0]);
    const R I_ac = inhib_pH<R>(Hr, p.pH_invK[1], p.pH_n[1], p.pH_nint[1]);
    const R I_h2 = inhib_pH<R>(Hr, p.pH_invK[2], p.pH_n[2], p.pH_nint[2]);
    const R sIN = (R)y[SIN];
    const R I_IN = sIN * frcp(sIN + (R)p.K_S_IN);                       // eq. 6
    const R nh3 = (R)c.K_a_IN * sIN * frcp((R)c.K_a_IN + Hr);
    const R I_nh3 = frcp((R)1 + nh3 * (R)p.inv_K_I_nh3);                // eq. 5
    const R I5 = I_aa * I_IN;

    R rho[19];
    rho[0] = a * (R)p.k_dis * (R)y[Xxc];
    rho[1] = a * (R)p.k_hyd_ch * (R)y[Xch];
    rho[2] = a * (R)p.k_hyd_pr * (R)y[Xpr];
    rho[3] = a * (R)p.k_hyd_li * (R)y[Xli];
    {
        const R s = (R)y[Ssu];
        rho[4] = a * (R)p.k_m_su * s * frcp((R)p.K_S_su + s) * (R)y[Xsu] * I5;
    }
    {
        const R s = (R)y[Saa];
        rho[5] = a * (R)p.k_m_aa * s * frcp((R)p.K_S_aa + s) * (R)y[Xaa] * I5;
    }
    const R sfa = (R)y[Sfa];
    const R b7 = a * (R)p.k_m_fa * sfa * frcp((R)p.K_S_fa + sfa) * (R)y[Xfa] * I5;
    const R sva = (R)y[Sva], sbu = (R)y[Sbu];
    const R isum = frcp(sva + sbu + (R)p.eps_c4);
    const R b8 = a * (R)p.k_m_c4 * sva * frcp((R)p.K_S_c4 + sva) * (R)y[Xc4] * sva * isum * I5;
    const R b9 = a * (R)p.k_m_c4 * sbu * frcp((R)p.K_S_c4 + sbu) * (R)y[Xc4] * sbu * isum * I5;
    const R spro = (R)y[Spro];
    const R b10 = a * (R)p.k_m_pro * spro * frcp((R)p.K_S_pro + spro) * (R)y[Xpro] * I5;
    {
        const R s = (R)y[Sac];
        rho[10] = a * (R)p.k_m_ac * s * frcp((R)p.K_S_ac + s) * (R)y[Xac] * I_ac * I_IN * I_nh3;
    }
    const R b12 = a * (R)p.k_m_h2 * (R)y[Xh2] * I_h2 * I_IN;
#pragma unroll
    for (int b = 0; b < 7; ++b) rho[12 + b] = a * (R)p.k_dec[b] * (R)y[Xsu + b];

    // eq. 8 (FP64) with the rate factors above
    H2Terms t;
    ADM1_H2_TERMS(t, inflow(ROW_SH2), rho, b7, b8, b9, b10, b12);
    t.kh = c.K_H_h2 * c.RT * y[Gh2];
    if (solve_Sh2(p, t, D, Sh2, iters)) return 1;
    if (alg_only) return 0;
    const R S = (R)Sh2;
    rho[6] = b7 * (R)p.K_I_h2_fa * frcp((R)p.K_I_h2_fa + S);
    const R ic4 = (R)p.K_I_h2_c4 * frcp((R)p.K_I_h2_c4 + S);
    rho[7] = b8 * ic4;
    rho[8] = b9 * ic4;
    rho[9] = b10 * (R)p.K_I_h2_pro * frcp((R)p.K_I_h2_pro + S);
    rho[11] = b12 * S * frcp((R)p.K_S_h2 + S);

    // liquid-gas transfer and headspace outflow
    const R kLa = (R)p.kLa;
    const R T8 = kLa * (S - (R)t.kh);
    const R T9 = kLa * ((R)y[Sch4] - (R)(c.K_H_ch4 * c.RT) * (R)y[Gch4]);
    const R co2 = (R)y[SIC] * Hr * frcp((R)c.K_a_co2 + Hr);
    const R T10 = kLa * (co2 - (R)(c.K_H_co2 * c.RT) * (R)y[Gco2]);
    const R P = (R)c.RT * ((R)y[Gh2] * (R)(1.0 / 16.0) + (R)y[Gch4] * (R)(1.0 / 64.0) +
                           (R)y[Gco2]) + (R)c.p_h2o;
    const R Patm = (R)p.P_atm;
    const R q = P > Patm ? (R)p.kp * (P - Patm) * P * (R)p.inv_P_atm : (R)0;

    // eq. 2 assembly
    const R Dr = (R)D;
#define ADM1_IN(k) ((R)inflow(state_row(k)) - Dr * (R)y[k])
    ADM1_ASSEMBLE_LIQUID(out, ADM1_IN, rho, R, T9, T10);
    {
        R sic = ADM1_IN(SIC) - T10, sin_ = ADM1_IN(SIN);
#pragma unroll
        for (int j = 0; j < 19; ++j) {
            sic += (R)p.nuIC[j] * rho[j];
            sin_ += (R)p.nuIN[j] * rho[j];
        }
        out(SIC, (double)sic);
        out(SIN, (double)sin_);
    }
#undef ADM1_IN
    const R ivg = (R)p.inv_vg;
    out(Gh2, (double)((T8 - q * (R)y[Gh2]) * ivg));
    out(Gch4, (double)((T9 - q * (R)y[Gch4]) * ivg));
    out(Gco2, (double)((T10 - q * (R)y[Gco2]) * ivg));
    return 0;
}

template <typename R>
__device__ __forceinline__ int rhs(const DevParams& p, const TConst& c, const double* y,
                                   double D, const double* sin, double& H, double& Sh2,
                                   double* f, int& iters)
{
    return rhs_in<R>(p, c, y, D, FeedInflow{D, sin}, H, Sh2,
                     [f](int k, double v) { f[k] = v; }, iters);
}

// ---------------------------------------------------------------------------
// Analytic partial derivatives of every rate in its inputs, at fixed
// (S_H+, S_h2), for the bordered Newton matrix.  FP64.
// ---------------------------------------------------------------------------
template <typename Y>
__device__ __forceinline__ void partials(const DevParams& p, const TConst& c, const Y& y,
                                         double H, double S, Partials& d)
{
    const double a = c.arr;
    // pH inhibition: dI/dH = -(n/H) I (1 - I)
    const double I_aa = inhib_pH<double>(H, p.pH_invK[0], p.pH_n[0], p.pH_nint[0]);
    const double I_ac = inhib_pH<double>(H, p.pH_invK[1], p.pH_n[1], p.pH_nint[1]);
    const double I_h2 = inhib_pH<double>(H, p.pH_invK[2], p.pH_n[2], p.pH_nint[2]);
    const double iH = 1.0 / H;
    const double dI_aa = -p.pH_n[0] * iH * I_aa * (1.0 - I_aa);
    const double dI_ac = -p.pH_n[1] * iH * I_ac * (1.0 - I_ac);
    const double dI_h2 = -p.pH_n[2] * iH * I_h2 * (1.0 - I_h2);
    // nitrogen limitation (eq. 6) and free-ammonia inhibition (eq. 5)
    const double iSIN = 1.0 / (y[SIN] + p.K_S_IN);
    const double I_IN = y[SIN] * iSIN, dI_IN = p.K_S_IN * iSIN * iSIN;
    const double iKIN = 1.0 / (c.K_a_IN + H);
    const double phiIN = c.K_a_IN * iKIN;
    const double nh3 = phiIN * y[SIN];
    const double I_nh3 = 1.0 / (1.0 + nh3 / p.K_I_nh3);
    const double dInh3_dnh3 = -I_nh3 * I_nh3 / p.K_I_nh3;
    const double dInh3_dSIN = dInh3_dnh3 * phiIN;
    const double dInh3_dH = dInh3_dnh3 * (-nh3 * iKIN);
    // hydrogen inhibitions (eq. 5) in S_h2: I = K/(K+S), dI/dS = -I/(K+S)
    const double ifa = 1.0 / (p.K_I_h2_fa + S), ic4 = 1.0 / (p.K_I_h2_c4 + S);
    const double ipr = 1.0 / (p.K_I_h2_pro + S);
    const double I_fa = p.K_I_h2_fa * ifa, I_c4 = p.K_I_h2_c4 * ic4, I_pr = p.K_I_h2_pro * ipr;

    d.J_dis_Xxc = a * p.k_dis;
    d.J_hch_Xch = a * p.k_hyd_ch;
    d.J_hpr_Xpr = a * p.k_hyd_pr;
    d.J_hli_Xli = a * p.k_hyd_li;

    // Monod uptake with the common pH/N inhibition I_aa I_IN (processes 5-7, 10)
    // rho = k_a M(s) X I_aa I_IN [Ih2]; M = s/(K+s), dM/ds = K/(K+s)^2
#define ADM1_MONOD(name, km, KS, sidx, xidx, extra, Sh2_factor_deriv)                      \
    {                                                                                    \
        const double s = y[sidx], X = y[xidx];                                           \
        const double iK = 1.0 / (KS + s);                                                \
        const double M = s * iK, dM = KS * iK * iK;                                      \
        const double kx = a * km * (extra);                                              \
        d.J_##name##_##sidx = kx * dM * X * I_aa * I_IN;                                 \
        d.J_##name##_##xidx = kx * M * I_aa * I_IN;                                      \
        d.J_##name##_SIN = kx * M * X * I_aa * dI_IN;                                    \
        d.J_##name##_H = kx * M * X * dI_aa * I_IN;                                      \
        Sh2_factor_deriv                                                                 \
    }
    ADM1_MONOD(su, p.k_m_su, p.K_S_su, Ssu, Xsu, 1.0, )
    ADM1_MONOD(aa, p.k_m_aa, p.K_S_aa, Saa, Xaa, 1.0, )
    ADM1_MONOD(fa, p.k_m_fa, p.K_S_fa, Sfa, Xfa, I_fa,
               d.J_fa_Sh2 = -(a * p.k_m_fa * M * X * I_aa * I_IN * I_fa) * ifa;)
    ADM1_MONOD(pro, p.k_m_pro, p.K_S_pro, Spro, Xpro, I_pr,
               d.J_pro_Sh2 = -(a * p.k_m_pro * M * X * I_aa * I_IN * I_pr) * ipr;)
#undef ADM1_MONOD

    // valerate / butyrate: rho = k_a M(s) X_c4 s/(S_va+S_bu+eps) I_aa I_IN I_c4
    {
        const double va = y[Sva], bu = y[Sbu], X = y[Xc4];
        const double iS = 1.0 / (va + bu + p.eps_c4);
        const double iKva = 1.0 / (p.K_S_c4 + va), iKbu = 1.0 / (p.K_S_c4 + bu);
        const double Mva = va * iKva, dMva = p.K_S_c4 * iKva * iKva;
        const double Mbu = bu * iKbu, dMbu = p.K_S_c4 * iKbu * iKbu;
        const double qva = va * iS, qbu = bu * iS;
        const double dqva_va = (bu + p.eps_c4) * iS * iS, dqva_bu = -va * iS * iS;
        const double dqbu_bu = (va + p.eps_c4) * iS * iS, dqbu_va = -bu * iS * iS;
        const double k = a * p.k_m_c4 * I_c4;
        const double Iab = I_aa * I_IN;
        const double r8 = k * Mva * X * qva * Iab, r9 = k * Mbu * X * qbu * Iab;
        d.J_va_Sva = k * X * Iab * (dMva * qva + Mva * dqva_va);
        d.J_va_Sbu = k * X * Iab * Mva * dqva_bu;
        d.J_va_Xc4 = k * Mva * qva * Iab;
        d.J_va_SIN = k * Mva * X * qva * I_aa * dI_IN;
        d.J_va_H = k * Mva * X * qva * dI_aa * I_IN;
        d.J_va_Sh2 = -r8 * ic4;
        d.J_bu_Sbu = k * X * Iab * (dMbu * qbu + Mbu * dqbu_bu);
        d.J_bu_Sva = k * X * Iab * Mbu * dqbu_va;
        d.J_bu_Xc4 = k * Mbu * qbu * Iab;
        d.J_bu_SIN = k * Mbu * X * qbu * I_aa * dI_IN;
        d.J_bu_H = k * Mbu * X * qbu * dI_aa * I_IN;
        d.J_bu_Sh2 = -r9 * ic4;
    }
    // acetate: rho = k_a M(S_ac) X_ac I_ac I_IN I_nh3
    {
        const double s = y[Sac], X = y[Xac];
        const double iK = 1.0 / (p.K_S_ac + s);
        const double M = s * iK, dM = p.K_S_ac * iK * iK;
        const double k = a * p.k_m_ac;
        d.J_ac_Sac = k * dM * X * I_ac * I_IN * I_nh3;
        d.J_ac_Xac = k * M * I_ac * I_IN * I_nh3;
        d.J_ac_SIN = k * M * X * I_ac * (dI_IN * I_nh3 + I_IN * dInh3_dSIN);
        d.J_ac_H = k * M * X * I_IN * (dI_ac * I_nh3 + I_ac * dInh3_dH);
    }
    // hydrogen: rho = k_a M(S_h2) X_h2 I_h2 I_IN
    {
        const double X = y[Xh2];
        const double iK = 1.0 / (p.K_S_h2 + S);
        const double M = S * iK, dM = p.K_S_h2 * iK * iK;
        const double k = a * p.k_m_h2;
        d.J_h2_Sh2 = k * dM * X * I_h2 * I_IN;
        d.J_h2_Xh2 = k * M * I_h2 * I_IN;
        d.J_h2_SIN = k * M * X * I_h2 * dI_IN;
        d.J_h2_H = k * M * X * dI_h2 * I_IN;
    }
    d.J_dsu_Xsu = a * p.k_dec[0];
    d.J_daa_Xaa = a * p.k_dec[1];
    d.J_dfa_Xfa = a * p.k_dec[2];
    d.J_dc4_Xc4 = a * p.k_dec[3];
    d.J_dpro_Xpro = a * p.k_dec[4];
    d.J_dac_Xac = a * p.k_dec[5];
    d.J_dh2_Xh2 = a * p.k_dec[6];

    // transfers: T8 = kLa (S_h2 - K_H RT G_h2), T9 likewise, T10 on S_co2
    d.J_T8_Sh2 = p.kLa;
    d.J_T8_Gh2 = -p.kLa * c.K_H_h2 * c.RT;
    d.J_T9_Sch4 = p.kLa;
    d.J_T9_Gch4 = -p.kLa * c.K_H_ch4 * c.RT;
    {
        const double iK = 1.0 / (c.K_a_co2 + H);
        const double phi = c.K_a_co2 * iK;
        d.J_T10_SIC = p.kLa * (1.0 - phi);
        d.J_T10_H = p.kLa * y[SIC] * phi * iK;
        d.J_T10_Gco2 = -p.kLa * c.K_H_co2 * c.RT;
    }
    // headspace outflow q(P) times each gas concentration
    {
        const double P = c.RT * (y[Gh2] * (1.0 / 16.0) + y[Gch4] * (1.0 / 64.0) + y[Gco2]) +
                         c.p_h2o;
        double q = 0.0, dq = 0.0;
        if (P > p.P_atm) {
            q = p.kp * (P - p.P_atm) * P / p.P_atm;
            dq = p.kp * (2.0 * P - p.P_atm) / p.P_atm;
        }
        const double dq1 = dq * c.RT * (1.0 / 16.0), dq2 = dq * c.RT * (1.0 / 64.0),
                     dq3 = dq * c.RT;
        d.J_QGh2_Gh2 = dq1 * y[Gh2] + q;
        d.J_QGh2_Gch4 = dq2 * y[Gh2];
        d.J_QGh2_Gco2 = dq3 * y[Gh2];
        d.J_QGch4_Gh2 = dq1 * y[Gch4];
        d.J_QGch4_Gch4 = dq2 * y[Gch4] + q;
        d.J_QGch4_Gco2 = dq3 * y[Gch4];
        d.J_QGco2_Gh2 = dq1 * y[Gco2];
        d.J_QGco2_Gch4 = dq2 * y[Gco2];
        d.J_QGco2_Gco2 = dq3 * y[Gco2] + q;
    }
    // eq. 7 gradient
    {
        const double iCO2 = 1.0 / (c.K_a_co2 + H);
        const double iac = 1.0 / (p.K_a_ac + H), ibu = 1.0 / (p.K_a_bu + H),
                     iva = 1.0 / (p.K_a_va + H), ipro = 1.0 / (p.K_a_pro + H);
        d.J_E7_Scat = 1.0;
        d.J_E7_San = -1.0;
        d.J_E7_SIN = 1.0 - phiIN;
        d.J_E7_SIC = -c.K_a_co2 * iCO2;
        d.J_E7_Sac = -p.K_a_ac * iac * (1.0 / 64.0);
        d.J_E7_Spro = -p.K_a_pro * ipro * (1.0 / 112.0);
        d.J_E7_Sbu = -p.K_a_bu * ibu * (1.0 / 160.0);
        d.J_E7_Sva = -p.K_a_va * iva * (1.0 / 208.0);
        d.J_E7_H = 1.0 + nh3 * iKIN + c.K_a_co2 * y[SIC] * iCO2 * iCO2 +
                   p.K_a_ac * y[Sac] * iac * iac * (1.0 / 64.0) +
                   p.K_a_pro * y[Spro] * ipro * ipro * (1.0 / 112.0) +
                   p.K_a_bu * y[Sbu] * ibu * ibu * (1.0 / 160.0) +
                   p.K_a_va * y[Sva] * iva * iva * (1.0 / 208.0) + c.K_w * iH * iH;
    }
}

}  // namespace adm1
