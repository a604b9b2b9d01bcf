/*
 * adm1_oracle.c -- ORACLE for the per-particle ADM1 reaction step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, serial FP64
 * reference that the HIP path is checked against.  Only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * What it computes (Kumar et al., "Introducing CHAD", arXiv 2311.08927):
 *   every particle is its own CSTR (sec. 2.3) whose ADM1 state obeys the mass
 *   balance of eq. 2 with the standard ADM1 rates (sec. 2.2), the inhibition
 *   forms of eqs. 3-6, and two algebraic equations that replace the stiff
 *   dynamics: the charge balance of eq. 7 (solved for S_H+) and the S_h2
 *   balance of eq. 8 (solved for S_h2).  The paper does not name its time
 *   integrator; this reference integrates the 28 differential entries with
 *   the Rosenbrock method Rodas4 (Hairer & Wanner, Solving ODEs II, sec. IV.7)
 *   under step-size control, the algebraic entries being re-solved at every
 *   right-hand-side evaluation.
 *
 * Plain by design: dense 28x28 Jacobian by complex-step differentiation
 * (Squire & Trapp 1998) through the algebraic solves, dense LU with partial
 * pivoting, one particle at a time.  Threads only split the particle list
 * into equal chunks, as in sec. 4.3.
 */
#ifndef ORC_COUNTED
#include <complex.h>
#endif
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The scalar of the right-hand side: double complex (the complex step of the
 * Jacobian), or an operation-counting type supplied by the includer
 * (count_ops.cpp defines ORC_COUNTED and cx before including this file). */
#ifndef ORC_COUNTED
typedef double complex cx;
#endif

/* ------------------------------------------------------------------------ */
/* State layout (35 entries).  Concentrations in kg COD/m3, except S_IC,     */
/* S_IN, S_cat, S_an, S_hco3, S_nh3 and G_co2 in kmol/m3.                    */
/* ------------------------------------------------------------------------ */
enum {
    S_SU, S_AA, S_FA, S_VA, S_BU, S_PRO, S_AC, S_H2, S_CH4, S_IC, S_IN, S_I,
    X_XC, X_CH, X_PR, X_LI, X_SU, X_AA, X_FA, X_C4, X_PRO, X_AC, X_H2, X_I,
    S_CAT, S_AN, S_VA_M, S_BU_M, S_PRO_M, S_AC_M, S_HCO3_M, S_NH3,
    G_H2, G_CH4, G_CO2, NX
};
#define NLIQ 26  /* entries 0..25 carry an inflow concentration */
#define ND 28    /* differential entries */
#define NPROC 19 /* biochemical processes */

/* the 28 differential entries, in the order of the integration vector */
static const int DIFF[ND] = {
    S_SU, S_AA, S_FA, S_VA, S_BU, S_PRO, S_AC, S_CH4, S_IC, S_IN, S_I,
    X_XC, X_CH, X_PR, X_LI, X_SU, X_AA, X_FA, X_C4, X_PRO, X_AC, X_H2, X_I,
    S_CAT, S_AN, G_H2, G_CH4, G_CO2
};

/* ------------------------------------------------------------------------ */
/* Parameters: filled by name from the parameter file by the binding.       */
/* ------------------------------------------------------------------------ */
#define ORC_PARAMS(X) \
    X(f_sI_xc) X(f_xI_xc) X(f_ch_xc) X(f_pr_xc) X(f_li_xc) \
    X(N_xc) X(N_I) X(N_aa) X(N_bac) \
    X(C_xc) X(C_sI) X(C_ch) X(C_pr) X(C_li) X(C_xI) X(C_su) X(C_aa) X(C_fa) \
    X(C_va) X(C_bu) X(C_pro) X(C_ac) X(C_bac) X(C_ch4) \
    X(f_fa_li) X(f_h2_su) X(f_bu_su) X(f_pro_su) X(f_ac_su) \
    X(f_h2_aa) X(f_va_aa) X(f_bu_aa) X(f_pro_aa) X(f_ac_aa) \
    X(f_ac_fa) X(f_h2_fa) X(f_pro_va) X(f_ac_va) X(f_h2_va) \
    X(f_ac_bu) X(f_h2_bu) X(f_ac_pro) X(f_h2_pro) \
    X(Y_su) X(Y_aa) X(Y_fa) X(Y_c4) X(Y_pro) X(Y_ac) X(Y_h2) \
    X(k_dis) X(k_hyd_ch) X(k_hyd_pr) X(k_hyd_li) \
    X(k_m_su) X(K_S_su) X(k_m_aa) X(K_S_aa) X(k_m_fa) X(K_S_fa) X(K_I_h2_fa) \
    X(k_m_c4) X(K_S_c4) X(K_I_h2_c4) X(k_m_pro) X(K_S_pro) X(K_I_h2_pro) \
    X(k_m_ac) X(K_S_ac) X(K_I_nh3) X(k_m_h2) X(K_S_h2) \
    X(k_dec_su) X(k_dec_aa) X(k_dec_fa) X(k_dec_c4) X(k_dec_pro) X(k_dec_ac) \
    X(k_dec_h2) X(K_S_IN) \
    X(pH_UL_aa) X(pH_LL_aa) X(pH_UL_ac) X(pH_LL_ac) X(pH_UL_h2) X(pH_LL_h2) \
    X(eps_c4) X(E_a) X(T_ref_kin) \
    X(R) X(T_base) X(K_w_base) X(dH_w) \
    X(K_a_va) X(K_a_bu) X(K_a_pro) X(K_a_ac) \
    X(K_a_co2_base) X(dH_a_co2) X(K_a_IN_base) X(dH_a_IN) \
    X(K_H_h2_base) X(dH_H_h2) X(K_H_ch4_base) X(dH_H_ch4) \
    X(K_H_co2_base) X(dH_H_co2) X(p_h2o_base) X(p_h2o_coef) \
    X(k_L_a) X(k_p_per_V_liq) X(V_gas_per_V_liq) X(P_atm)

typedef struct {
#define ORC_DECL(n) double n;
    ORC_PARAMS(ORC_DECL)
#undef ORC_DECL
    /* A model description's Petersen matrix (organic rows; the S_IC and S_IN
     * rows are closures) and carbon / nitrogen contents, evaluated by the
     * binding from the description file; used instead of the built-in
     * standard ADM1 formulas below when model_set is nonzero. */
    double model_nu[NLIQ][NPROC];
    double model_C[NLIQ], model_N[NLIQ];
    double model_set;
} orc_params;

static const char orc_names[] =
#define ORC_NAME(n) #n ","
    ORC_PARAMS(ORC_NAME)
#undef ORC_NAME
    ;

const char *orc_param_names(void) { return orc_names; }
#define ORC_ONE(n) +1
int orc_param_count(void) { return 0 ORC_PARAMS(ORC_ONE); }
#undef ORC_ONE
/* size of the parameter block in doubles; the model fields follow the named
 * parameters: model_nu at orc_param_count(), then model_C, model_N,
 * model_set */
int orc_params_doubles(void) { return (int)(sizeof(orc_params) / sizeof(double)); }

/* Integration options (sec. 2.3 leaves them open; see the readings). */
typedef struct {
    double rtol;
    double atol[ND];
    int max_steps;     /* attempted steps per interval */
    double newton_tol; /* relative step tolerance of the algebraic solves */
    int newton_maxit;
} orc_opts;

/* ------------------------------------------------------------------------ */
/* Temperature-dependent constants.  The paper fixes T per case (Tables 1-2).*/
/* Van't Hoff for K_w, K_a,co2, K_a,IN and Henry constants; an Arrhenius    */
/* factor on the kinetic rate constants (a reading: the paper runs at one   */
/* temperature).                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double RT, K_w, K_a_co2, K_a_IN, K_H_h2, K_H_ch4, K_H_co2, p_h2o, arr;
} orc_tconst;

static orc_tconst orc_tconsts(const orc_params *p, double T);

/* Multiple phases (sec. 5: particles of several kinds, such as sediments or
 * inert matter): a phase scales every biochemical rate of the particle by
 * its kinetic factor kin (0: an inert phase, reactions off), while dilution
 * and the liquid-gas transfers act as in any particle.  Every rate of eq. 2
 * carries the temperature factor arr as a multiplier, so the phase factor
 * is applied there. */
static orc_tconst phase_tconsts(const orc_params *p, double T, double kin)
{
    orc_tconst c = orc_tconsts(p, T);
    c.arr *= kin;
    return c;
}

static orc_tconst orc_tconsts(const orc_params *p, double T)
{
    orc_tconst c;
    const double R100 = 100.0 * p->R;         /* J/(mol K) */
    const double vh = 1.0 / p->T_base - 1.0 / T;
    c.RT = p->R * T;
    c.K_w = p->K_w_base * exp(p->dH_w / R100 * vh);
    c.K_a_co2 = p->K_a_co2_base * exp(p->dH_a_co2 / R100 * vh);
    c.K_a_IN = p->K_a_IN_base * exp(p->dH_a_IN / R100 * vh);
    c.K_H_h2 = p->K_H_h2_base * exp(p->dH_H_h2 / R100 * vh);
    c.K_H_ch4 = p->K_H_ch4_base * exp(p->dH_H_ch4 / R100 * vh);
    c.K_H_co2 = p->K_H_co2_base * exp(p->dH_H_co2 / R100 * vh);
    c.p_h2o = p->p_h2o_base * exp(p->p_h2o_coef * vh);
    c.arr = exp(p->E_a / R100 * (1.0 / p->T_ref_kin - 1.0 / T));
    return c;
}

void orc_tconst_export(const orc_params *p, double T, double out[9])
{
    orc_tconst c = orc_tconsts(p, T);
    out[0] = c.RT; out[1] = c.K_w; out[2] = c.K_a_co2; out[3] = c.K_a_IN;
    out[4] = c.K_H_h2; out[5] = c.K_H_ch4; out[6] = c.K_H_co2; out[7] = c.p_h2o;
    out[8] = c.arr;
}

/* ------------------------------------------------------------------------ */
/* Petersen (stoichiometry) matrix nu[i][j] of eq. 2, rows = entries 0..25,  */
/* columns = the 19 processes: disintegration, 3 hydrolyses, 8 uptakes,      */
/* 7 decays.  S_IC and S_IN rows close carbon and nitrogen.                 */
/* ------------------------------------------------------------------------ */
static void carbon_nitrogen(const orc_params *p, double C[NLIQ], double N[NLIQ])
{
    if (p->model_set != 0.0) {
        for (int i = 0; i < NLIQ; i++) { C[i] = p->model_C[i]; N[i] = p->model_N[i]; }
        return;
    }
    for (int i = 0; i < NLIQ; i++) { C[i] = 0.0; N[i] = 0.0; }
    C[S_SU] = p->C_su; C[S_AA] = p->C_aa; C[S_FA] = p->C_fa; C[S_VA] = p->C_va;
    C[S_BU] = p->C_bu; C[S_PRO] = p->C_pro; C[S_AC] = p->C_ac; C[S_CH4] = p->C_ch4;
    C[S_I] = p->C_sI; C[X_XC] = p->C_xc; C[X_CH] = p->C_ch; C[X_PR] = p->C_pr;
    C[X_LI] = p->C_li; C[X_I] = p->C_xI;
    for (int i = X_SU; i <= X_H2; i++) C[i] = p->C_bac;
    N[S_AA] = p->N_aa; N[S_I] = p->N_I; N[X_XC] = p->N_xc; N[X_PR] = p->N_aa;
    N[X_I] = p->N_I;
    for (int i = X_SU; i <= X_H2; i++) N[i] = p->N_bac;
}

static void petersen(const orc_params *p, double nu[NLIQ][NPROC])
{
    memset(nu, 0, sizeof(double) * NLIQ * NPROC);
    if (p->model_set != 0.0) {
        memcpy(nu, p->model_nu, sizeof(double) * NLIQ * NPROC);
        goto closures;
    }
    /* 1 disintegration */
    nu[X_XC][0] = -1.0; nu[S_I][0] = p->f_sI_xc; nu[X_CH][0] = p->f_ch_xc;
    nu[X_PR][0] = p->f_pr_xc; nu[X_LI][0] = p->f_li_xc; nu[X_I][0] = p->f_xI_xc;
    /* 2-4 hydrolysis */
    nu[X_CH][1] = -1.0; nu[S_SU][1] = 1.0;
    nu[X_PR][2] = -1.0; nu[S_AA][2] = 1.0;
    nu[X_LI][3] = -1.0; nu[S_SU][3] = 1.0 - p->f_fa_li; nu[S_FA][3] = p->f_fa_li;
    /* 5 uptake of sugars */
    nu[S_SU][4] = -1.0;
    nu[S_BU][4] = (1.0 - p->Y_su) * p->f_bu_su;
    nu[S_PRO][4] = (1.0 - p->Y_su) * p->f_pro_su;
    nu[S_AC][4] = (1.0 - p->Y_su) * p->f_ac_su;
    nu[S_H2][4] = (1.0 - p->Y_su) * p->f_h2_su;
    nu[X_SU][4] = p->Y_su;
    /* 6 uptake of amino acids */
    nu[S_AA][5] = -1.0;
    nu[S_VA][5] = (1.0 - p->Y_aa) * p->f_va_aa;
    nu[S_BU][5] = (1.0 - p->Y_aa) * p->f_bu_aa;
    nu[S_PRO][5] = (1.0 - p->Y_aa) * p->f_pro_aa;
    nu[S_AC][5] = (1.0 - p->Y_aa) * p->f_ac_aa;
    nu[S_H2][5] = (1.0 - p->Y_aa) * p->f_h2_aa;
    nu[X_AA][5] = p->Y_aa;
    /* 7 uptake of LCFA */
    nu[S_FA][6] = -1.0;
    nu[S_AC][6] = (1.0 - p->Y_fa) * p->f_ac_fa;
    nu[S_H2][6] = (1.0 - p->Y_fa) * p->f_h2_fa;
    nu[X_FA][6] = p->Y_fa;
    /* 8 uptake of valerate */
    nu[S_VA][7] = -1.0;
    nu[S_PRO][7] = (1.0 - p->Y_c4) * p->f_pro_va;
    nu[S_AC][7] = (1.0 - p->Y_c4) * p->f_ac_va;
    nu[S_H2][7] = (1.0 - p->Y_c4) * p->f_h2_va;
    nu[X_C4][7] = p->Y_c4;
    /* 9 uptake of butyrate */
    nu[S_BU][8] = -1.0;
    nu[S_AC][8] = (1.0 - p->Y_c4) * p->f_ac_bu;
    nu[S_H2][8] = (1.0 - p->Y_c4) * p->f_h2_bu;
    nu[X_C4][8] = p->Y_c4;
    /* 10 uptake of propionate */
    nu[S_PRO][9] = -1.0;
    nu[S_AC][9] = (1.0 - p->Y_pro) * p->f_ac_pro;
    nu[S_H2][9] = (1.0 - p->Y_pro) * p->f_h2_pro;
    nu[X_PRO][9] = p->Y_pro;
    /* 11 uptake of acetate */
    nu[S_AC][10] = -1.0; nu[S_CH4][10] = 1.0 - p->Y_ac; nu[X_AC][10] = p->Y_ac;
    /* 12 uptake of hydrogen */
    nu[S_H2][11] = -1.0; nu[S_CH4][11] = 1.0 - p->Y_h2; nu[X_H2][11] = p->Y_h2;
    /* 13-19 decay of the seven biomasses into composites */
    for (int b = 0; b < 7; b++) { nu[X_SU + b][12 + b] = -1.0; nu[X_XC][12 + b] = 1.0; }

closures:;
    /* carbon and nitrogen closure: inorganic C and N take up whatever the
     * organic entries release, so C and N are conserved by every process */
    double C[NLIQ], N[NLIQ];
    carbon_nitrogen(p, C, N);
    for (int j = 0; j < NPROC; j++) {
        double sc = 0.0, sn = 0.0;
        for (int i = 0; i < NLIQ; i++) {
            if (i == S_IC || i == S_IN) continue;
            sc += C[i] * nu[i][j];
            sn += N[i] * nu[i][j];
        }
        nu[S_IC][j] = -sc;
        nu[S_IN][j] = -sn;
    }
}

void orc_petersen(const orc_params *p, double *out /* [26][19] */)
{
    double nu[NLIQ][NPROC];
    petersen(p, nu);
    memcpy(out, nu, sizeof(nu));
}

void orc_contents(const orc_params *p, double *C_out, double *N_out)
{
    carbon_nitrogen(p, C_out, N_out);
}

/* Returns 0 when every process conserves COD (the COD-bearing entries sum
 * to zero), -1 otherwise. */
int orc_check_params(const orc_params *p)
{
    double nu[NLIQ][NPROC];
    petersen(p, nu);
    static const int cod[] = {S_SU, S_AA, S_FA, S_VA, S_BU, S_PRO, S_AC, S_H2, S_CH4,
                              S_I, X_XC, X_CH, X_PR, X_LI, X_SU, X_AA, X_FA, X_C4,
                              X_PRO, X_AC, X_H2, X_I};
    for (int j = 0; j < NPROC; j++) {
        double s = 0.0;
        for (size_t k = 0; k < sizeof(cod) / sizeof(cod[0]); k++) s += nu[cod[k]][j];
        if (fabs(s) > 1e-12) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Inhibition functions, eqs. 3-6.                                          */
/* ------------------------------------------------------------------------ */
/* eq. 5: non-competitive inhibition */
static cx inhib_noncomp(cx S, double K) { return 1.0 / (1.0 + S / K); }
/* eq. 6: substrate limitation */
static cx inhib_limit(cx S, double K) { return S / (S + K); }
/* eqs. 3-4, Hill form written in S_H+ (reading: the half point sits at the
 * mean of the lower and upper pH limits, exponent 3/(UL-LL)) */
static cx inhib_pH(cx SH, double pH_LL, double pH_UL)
{
    const double n = 3.0 / (pH_UL - pH_LL);
    const double K = pow(10.0, -0.5 * (pH_LL + pH_UL));
    const double Kn = pow(K, n);
    return Kn / (cpow(SH, n) + Kn);
}

double orc_inhib(int kind, double S, double a, double b)
{
    if (kind == 0) return creal(inhib_noncomp(S, a));
    if (kind == 1) return creal(inhib_limit(S, a));
    return creal(inhib_pH(S, a, b));
}

/* ------------------------------------------------------------------------ */
/* Eq. 7: charge balance E(S_H+) and its derivative in S_H+.                */
/* The ions are the equilibrium fractions of their totals.                  */
/* ------------------------------------------------------------------------ */
static cx charge_balance(const orc_params *p, const orc_tconst *c, const cx *x, cx H,
                         cx *dE)
{
    const cx nh3 = c->K_a_IN * x[S_IN] / (c->K_a_IN + H);
    const cx nh4 = x[S_IN] - nh3;
    const cx hco3 = c->K_a_co2 * x[S_IC] / (c->K_a_co2 + H);
    const cx ac = p->K_a_ac * x[S_AC] / (p->K_a_ac + H);
    const cx pro = p->K_a_pro * x[S_PRO] / (p->K_a_pro + H);
    const cx bu = p->K_a_bu * x[S_BU] / (p->K_a_bu + H);
    const cx va = p->K_a_va * x[S_VA] / (p->K_a_va + H);
    const cx E = x[S_CAT] + nh4 + H - hco3 - ac / 64.0 - pro / 112.0 - bu / 160.0
                 - va / 208.0 - c->K_w / H - x[S_AN];
    if (dE) {
        *dE = 1.0 + c->K_a_IN * x[S_IN] / ((c->K_a_IN + H) * (c->K_a_IN + H))
              + c->K_a_co2 * x[S_IC] / ((c->K_a_co2 + H) * (c->K_a_co2 + H))
              + p->K_a_ac * x[S_AC] / (64.0 * (p->K_a_ac + H) * (p->K_a_ac + H))
              + p->K_a_pro * x[S_PRO] / (112.0 * (p->K_a_pro + H) * (p->K_a_pro + H))
              + p->K_a_bu * x[S_BU] / (160.0 * (p->K_a_bu + H) * (p->K_a_bu + H))
              + p->K_a_va * x[S_VA] / (208.0 * (p->K_a_va + H) * (p->K_a_va + H))
              + c->K_w / (H * H);
    }
    return E;
}

/* Safeguarded Newton for eq. 7.  E is strictly increasing in S_H+ with
 * E -> -inf at 0+ and +inf at +inf (for non-negative totals), so the root is
 * unique: bracket it, then take Newton steps that stay inside the bracket,
 * bisecting (geometrically) otherwise.  A final Newton step carries the
 * derivative part of a complex-step perturbation.  Returns 0 on success. */
static int solve_SH(const orc_params *p, const orc_opts *o, const orc_tconst *c,
                    const cx *x, double guess, cx *H_out, int *iters)
{
    double lo = (guess > 0.0 && isfinite(guess)) ? guess : 1e-7;
    double hi = lo;
    int k = 0;
    while (creal(charge_balance(p, c, x, lo, NULL)) > 0.0) {
        lo *= 0.01;
        if (lo < 1e-30 || ++k > 60) return -1;
    }
    while (creal(charge_balance(p, c, x, hi, NULL)) < 0.0) {
        hi *= 100.0;
        if (hi > 1e10 || ++k > 60) return -1;
    }
    cx H = (guess >= lo && guess <= hi) ? guess : sqrt(lo * hi);
    int it = 0, done = 0;
    while (!done) {
        if (++it > o->newton_maxit) return -1;
        cx dE;
        const cx E = charge_balance(p, c, x, H, &dE);
        if (!isfinite(creal(E)) || !isfinite(creal(dE))) return -1;
        if (creal(E) < 0.0) lo = creal(H); else hi = creal(H);
        cx Hn = H - E / dE;
        if (!(creal(Hn) > lo && creal(Hn) < hi)) Hn = sqrt(lo * hi);
        if (fabs(creal(Hn) - creal(H)) <= o->newton_tol * fabs(creal(Hn))) done = 1;
        H = Hn;
    }
    cx dE;
    const cx E = charge_balance(p, c, x, H, &dE);
    H = H - E / dE;
    *H_out = H;
    if (iters) *iters += it;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Kinetic rates rho_j (19) and liquid-gas transfers (3), per m3 liquid.    */
/* x must hold S_H2 in its slot; H is S_H+.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    cx rho[NPROC];
    cx rhoT[3];        /* h2, ch4, co2 transfer, kg COD or kmol per m3 per d */
    cx q_per_V;        /* gas flow per m3 liquid, 1/d */
    cx p_h2, p_ch4, p_co2, P_gas;
} orc_rates_t;

static void rates(const orc_params *p, const orc_tconst *c, const cx *x, cx H,
                  orc_rates_t *r)
{
    const double a = c->arr;
    const cx IpH_aa = inhib_pH(H, p->pH_LL_aa, p->pH_UL_aa);
    const cx IpH_ac = inhib_pH(H, p->pH_LL_ac, p->pH_UL_ac);
    const cx IpH_h2 = inhib_pH(H, p->pH_LL_h2, p->pH_UL_h2);
    const cx I_IN = inhib_limit(x[S_IN], p->K_S_IN);
    const cx I_h2_fa = inhib_noncomp(x[S_H2], p->K_I_h2_fa);
    const cx I_h2_c4 = inhib_noncomp(x[S_H2], p->K_I_h2_c4);
    const cx I_h2_pro = inhib_noncomp(x[S_H2], p->K_I_h2_pro);
    const cx nh3 = c->K_a_IN * x[S_IN] / (c->K_a_IN + H);
    const cx I_nh3 = inhib_noncomp(nh3, p->K_I_nh3);
    const cx I5 = IpH_aa * I_IN;

    r->rho[0] = a * p->k_dis * x[X_XC];
    r->rho[1] = a * p->k_hyd_ch * x[X_CH];
    r->rho[2] = a * p->k_hyd_pr * x[X_PR];
    r->rho[3] = a * p->k_hyd_li * x[X_LI];
    r->rho[4] = a * p->k_m_su * x[S_SU] / (p->K_S_su + x[S_SU]) * x[X_SU] * I5;
    r->rho[5] = a * p->k_m_aa * x[S_AA] / (p->K_S_aa + x[S_AA]) * x[X_AA] * I5;
    r->rho[6] = a * p->k_m_fa * x[S_FA] / (p->K_S_fa + x[S_FA]) * x[X_FA] * I5 * I_h2_fa;
    r->rho[7] = a * p->k_m_c4 * x[S_VA] / (p->K_S_c4 + x[S_VA]) * x[X_C4]
                * x[S_VA] / (x[S_BU] + x[S_VA] + p->eps_c4) * I5 * I_h2_c4;
    r->rho[8] = a * p->k_m_c4 * x[S_BU] / (p->K_S_c4 + x[S_BU]) * x[X_C4]
                * x[S_BU] / (x[S_BU] + x[S_VA] + p->eps_c4) * I5 * I_h2_c4;
    r->rho[9] = a * p->k_m_pro * x[S_PRO] / (p->K_S_pro + x[S_PRO]) * x[X_PRO] * I5
                * I_h2_pro;
    r->rho[10] = a * p->k_m_ac * x[S_AC] / (p->K_S_ac + x[S_AC]) * x[X_AC] * IpH_ac
                 * I_IN * I_nh3;
    r->rho[11] = a * p->k_m_h2 * x[S_H2] / (p->K_S_h2 + x[S_H2]) * x[X_H2] * IpH_h2 * I_IN;
    r->rho[12] = a * p->k_dec_su * x[X_SU];
    r->rho[13] = a * p->k_dec_aa * x[X_AA];
    r->rho[14] = a * p->k_dec_fa * x[X_FA];
    r->rho[15] = a * p->k_dec_c4 * x[X_C4];
    r->rho[16] = a * p->k_dec_pro * x[X_PRO];
    r->rho[17] = a * p->k_dec_ac * x[X_AC];
    r->rho[18] = a * p->k_dec_h2 * x[X_H2];

    /* partial pressures: 16 and 64 kg COD per kmol for h2 and ch4 */
    r->p_h2 = x[G_H2] * c->RT / 16.0;
    r->p_ch4 = x[G_CH4] * c->RT / 64.0;
    r->p_co2 = x[G_CO2] * c->RT;
    r->P_gas = r->p_h2 + r->p_ch4 + r->p_co2 + c->p_h2o;
    const cx co2 = x[S_IC] - c->K_a_co2 * x[S_IC] / (c->K_a_co2 + H);
    r->rhoT[0] = p->k_L_a * (x[S_H2] - 16.0 * c->K_H_h2 * r->p_h2);
    r->rhoT[1] = p->k_L_a * (x[S_CH4] - 64.0 * c->K_H_ch4 * r->p_ch4);
    r->rhoT[2] = p->k_L_a * (co2 - c->K_H_co2 * r->p_co2);
    /* gas outflow through the headspace valve, zero below ambient pressure */
    if (creal(r->P_gas) > p->P_atm)
        r->q_per_V = p->k_p_per_V_liq * (r->P_gas - p->P_atm) * r->P_gas / p->P_atm;
    else
        r->q_per_V = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 8: S_h2 balance E(S_h2) and its derivative (analytic: only the three  */
/* eq.-5 hydrogen inhibitions, the hydrogen-uptake Monod term, transfer and */
/* dilution depend on S_h2).                                                 */
/* ------------------------------------------------------------------------ */
static cx h2_balance(const orc_params *p, const orc_tconst *c, cx *x, cx H, double D,
                     double s_in_h2, const double nu[NLIQ][NPROC], cx *dE)
{
    orc_rates_t r;
    rates(p, c, x, H, &r);
    cx E = D * (s_in_h2 - x[S_H2]) - r.rhoT[0];
    for (int j = 0; j < NPROC; j++) E += nu[S_H2][j] * r.rho[j];
    if (dE) {
        const cx S = x[S_H2];
        cx d = -D - p->k_L_a;
        d += nu[S_H2][6] * r.rho[6] * (-1.0 / (p->K_I_h2_fa + S));
        d += nu[S_H2][7] * r.rho[7] * (-1.0 / (p->K_I_h2_c4 + S));
        d += nu[S_H2][8] * r.rho[8] * (-1.0 / (p->K_I_h2_c4 + S));
        d += nu[S_H2][9] * r.rho[9] * (-1.0 / (p->K_I_h2_pro + S));
        /* rho_12 = k X I * S/(K+S): derivative k X I * K/(K+S)^2 */
        const cx IpH_h2 = inhib_pH(H, p->pH_LL_h2, p->pH_UL_h2);
        const cx I_IN = inhib_limit(x[S_IN], p->K_S_IN);
        d += nu[S_H2][11] * c->arr * p->k_m_h2 * x[X_H2] * IpH_h2 * I_IN * p->K_S_h2
             / ((p->K_S_h2 + S) * (p->K_S_h2 + S));
        *dE = d;
    }
    return E;
}

/* Safeguarded Newton for eq. 8.  E is strictly decreasing in S_h2 on
 * (-Kmin, inf), Kmin the smallest half-saturation/inhibition constant of
 * the terms above; for non-negative states E(0) >= 0, so the root is unique
 * and non-negative.  The upper end of the bracket follows from dropping the
 * (decreasing) production terms' dependence on S_h2. */
static int solve_Sh2(const orc_params *p, const orc_opts *o, const orc_tconst *c, cx *x,
                     cx H, double D, double s_in_h2, const double nu[NLIQ][NPROC],
                     double guess, int *iters)
{
    double Kmin = p->K_S_h2;
    if (p->K_I_h2_fa < Kmin) Kmin = p->K_I_h2_fa;
    if (p->K_I_h2_c4 < Kmin) Kmin = p->K_I_h2_c4;
    if (p->K_I_h2_pro < Kmin) Kmin = p->K_I_h2_pro;
    double lo = 0.0;
    x[S_H2] = 0.0;
    double E0 = creal(h2_balance(p, c, x, H, D, s_in_h2, nu, NULL));
    if (!isfinite(E0)) return -1;
    if (E0 < 0.0) {
        lo = -0.5 * Kmin;
        x[S_H2] = lo;
        if (creal(h2_balance(p, c, x, H, D, s_in_h2, nu, NULL)) < 0.0) return -1;
    }
    /* production at S_h2 = 0 bounds the production for S_h2 > 0 */
    double P0 = 0.0;
    {
        orc_rates_t r;
        x[S_H2] = 0.0;
        rates(p, c, x, H, &r);
        for (int j = 0; j < NPROC; j++)
            if (nu[S_H2][j] > 0.0) P0 += nu[S_H2][j] * creal(r.rho[j]);
    }
    const double pT = 16.0 * c->K_H_h2 * creal(x[G_H2]) * c->RT / 16.0;
    const double den = D + p->k_L_a;
    double hi = den > 0.0 ? (D * s_in_h2 + (P0 > 0.0 ? P0 : 0.0) +
                             p->k_L_a * (pT > 0.0 ? pT : 0.0)) / den
                          : Kmin;
    if (hi <= lo) hi = lo + Kmin;
    int k = 0;
    for (;;) {
        x[S_H2] = hi;
        const double Ehi = creal(h2_balance(p, c, x, H, D, s_in_h2, nu, NULL));
        if (!isfinite(Ehi)) return -1;
        if (Ehi <= 0.0) break;
        hi = 2.0 * hi + Kmin;
        if (++k > 200) return -1;
    }
    cx S = (guess > lo && guess < hi) ? guess : 0.5 * (lo + hi);
    int it = 0, done = 0;
    while (!done) {
        if (++it > o->newton_maxit) return -1;
        x[S_H2] = S;
        cx dE;
        const cx E = h2_balance(p, c, x, H, D, s_in_h2, nu, &dE);
        if (!isfinite(creal(E)) || !isfinite(creal(dE))) return -1;
        if (creal(E) > 0.0) lo = creal(S); else hi = creal(S);
        cx Sn = S - E / dE;
        if (!(creal(Sn) > lo && creal(Sn) < hi)) Sn = 0.5 * (lo + hi);
        if (fabs(creal(Sn) - creal(S)) <= o->newton_tol * fabs(creal(Sn)) + 1e-30) done = 1;
        S = Sn;
    }
    x[S_H2] = S;
    cx dE;
    const cx E = h2_balance(p, c, x, H, D, s_in_h2, nu, &dE);
    S = S - E / dE;
    x[S_H2] = S;
    if (iters) *iters += it;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of the 28 differential entries (eq. 2 for the liquid,    */
/* headspace balance for the gas), with the algebraic entries re-solved.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_params *p;
    const orc_opts *o;
    orc_tconst c;
    double nu[NLIQ][NPROC];
    double D;
    double s_in[NLIQ];
    double H_guess;   /* warm start of the eq.-7 solve */
    double Sh2_guess; /* warm start of the eq.-8 solve */
    int newton_iters;
} orc_model;

/* Fills x[35] (algebraic entries included) from the 28-vector y. */
static int algebraic(orc_model *m, const cx *y, cx *x, cx *H_out)
{
    for (int i = 0; i < NX; i++) x[i] = 0.0;
    for (int k = 0; k < ND; k++) x[DIFF[k]] = y[k];
    cx H;
    if (solve_SH(m->p, m->o, &m->c, x, m->H_guess, &H, &m->newton_iters)) return -1;
    if (solve_Sh2(m->p, m->o, &m->c, x, H, m->D, m->s_in[S_H2], m->nu, m->Sh2_guess,
                  &m->newton_iters))
        return -1;
    const orc_params *p = m->p;
    x[S_VA_M] = p->K_a_va * x[S_VA] / (p->K_a_va + H);
    x[S_BU_M] = p->K_a_bu * x[S_BU] / (p->K_a_bu + H);
    x[S_PRO_M] = p->K_a_pro * x[S_PRO] / (p->K_a_pro + H);
    x[S_AC_M] = p->K_a_ac * x[S_AC] / (p->K_a_ac + H);
    x[S_HCO3_M] = m->c.K_a_co2 * x[S_IC] / (m->c.K_a_co2 + H);
    x[S_NH3] = m->c.K_a_IN * x[S_IN] / (m->c.K_a_IN + H);
    *H_out = H;
    /* the next solve starts from these roots */
    m->H_guess = creal(H);
    m->Sh2_guess = creal(x[S_H2]);
    return 0;
}

static int rhs(orc_model *m, const cx *y, cx *f, cx *H_out)
{
    cx x[NX], H;
    if (algebraic(m, y, x, &H)) return -1;
    orc_rates_t r;
    rates(m->p, &m->c, x, H, &r);
    cx dx[NX];
    for (int i = 0; i < NX; i++) dx[i] = 0.0;
    for (int i = 0; i < NLIQ; i++) {
        cx s = m->D * (m->s_in[i] - x[i]);
        for (int j = 0; j < NPROC; j++) s += m->nu[i][j] * r.rho[j];
        dx[i] = s;
    }
    dx[S_CH4] -= r.rhoT[1];
    dx[S_IC] -= r.rhoT[2];
    const double vg = m->p->V_gas_per_V_liq;
    const cx q_over_Vg = r.q_per_V / vg;
    dx[G_H2] = -q_over_Vg * x[G_H2] + r.rhoT[0] / vg;
    dx[G_CH4] = -q_over_Vg * x[G_CH4] + r.rhoT[1] / vg;
    dx[G_CO2] = -q_over_Vg * x[G_CO2] + r.rhoT[2] / vg;
    for (int k = 0; k < ND; k++) f[k] = dx[DIFF[k]];
    if (H_out) *H_out = H;
    return 0;
}

static int rhs_real(orc_model *m, const double *y, double *f)
{
    cx yc[ND], fc[ND], H;
    for (int k = 0; k < ND; k++) yc[k] = y[k];
    if (rhs(m, yc, fc, &H)) return -1;
    for (int k = 0; k < ND; k++) f[k] = creal(fc[k]);
    return 0;
}

/* Total derivative df/dy (28x28, row-major) by complex-step differentiation:
 * column k is Im f(y + i h e_k) / h.  The algebraic solves run in complex
 * arithmetic, so the implicit dependence of S_H+ and S_h2 on y is included
 * exactly (to rounding). */
static int jacobian(orc_model *m, const double *y, double *J)
{
    const double h = 1e-40;
    for (int k = 0; k < ND; k++) {
        cx yc[ND], fc[ND];
        for (int i = 0; i < ND; i++) yc[i] = y[i];
        yc[k] += I * h;
        if (rhs(m, yc, fc, NULL)) return -1;
        for (int i = 0; i < ND; i++) J[i * ND + k] = cimag(fc[i]) / h;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (Doolittle), and the matching solve.      */
/* ------------------------------------------------------------------------ */
static int lu_factor(double *A, int n, int *piv)
{
    for (int k = 0; k < n; k++) {
        int pr = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); pr = i; }
        piv[k] = pr;
        if (!(best > 0.0) || !isfinite(best)) return -1;
        if (pr != k)
            for (int j = 0; j < n; j++) {
                double t = A[k * n + j]; A[k * n + j] = A[pr * n + j]; A[pr * n + j] = t;
            }
        for (int i = k + 1; i < n; i++) {
            A[i * n + k] /= A[k * n + k];
            const double l = A[i * n + k];
            for (int j = k + 1; j < n; j++) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

static void lu_solve(const double *A, int n, const int *piv, double *b)
{
    for (int k = 0; k < n; k++)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < n; i++)
        for (int k = 0; k < i; k++) b[i] -= A[i * n + k] * b[k];
    for (int i = n - 1; i >= 0; i--) {
        for (int k = i + 1; k < n; k++) b[i] -= A[i * n + k] * b[k];
        b[i] /= A[i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Rodas4 (Hairer & Wanner, sec. IV.7), in the transformed variables         */
/* u_i = sum_j gamma_ij k_j:                                                 */
/*   (I/(gamma h) - J) u_i = f(y0 + sum_j a_ij u_j) + sum_j (c_ij / h) u_j   */
/* Stiffly accurate: the embedded solution is y0 + sum a_5j u_j + u_5, the   */
/* solution adds u_6, and u_6 is the local error estimate.                   */
/* ------------------------------------------------------------------------ */
static const double R4_GAMMA = 0.25;
static const double R4_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0},
};
static const double R4_C[6][5] = {
    {0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054},
};

void orc_rodas4_tableau(double *gamma, double *A /*6x5*/, double *C /*6x5*/)
{
    *gamma = R4_GAMMA;
    memcpy(A, R4_A, sizeof(R4_A));
    memcpy(C, R4_C, sizeof(R4_C));
}

/* One Rodas4 step of size h from y0.  Writes y1 and the scaled RMS error
 * (sc_i = atol_i + rtol max(|y0_i|, |y1_i|)).  Returns -1 when an algebraic
 * solve or the factorisation fails inside the step. */
static int rodas4_step(orc_model *m, const double *y0, double h, double *y1, double *err)
{
    double J[ND * ND], W[ND * ND], u[6][ND], arg[ND], f[ND];
    int piv[ND];
    if (jacobian(m, y0, J)) return -1;
    for (int i = 0; i < ND; i++)
        for (int k = 0; k < ND; k++)
            W[i * ND + k] = (i == k ? 1.0 / (R4_GAMMA * h) : 0.0) - J[i * ND + k];
    if (lu_factor(W, ND, piv)) return -1;
    for (int s = 0; s < 6; s++) {
        for (int i = 0; i < ND; i++) {
            double a = y0[i];
            for (int j = 0; j < s; j++) a += R4_A[s][j] * u[j][i];
            arg[i] = a;
        }
        if (rhs_real(m, arg, f)) return -1;
        for (int i = 0; i < ND; i++) {
            double b = f[i];
            for (int j = 0; j < s; j++) b += R4_C[s][j] / h * u[j][i];
            u[s][i] = b;
        }
        lu_solve(W, ND, piv, u[s]);
    }
    double e = 0.0;
    for (int i = 0; i < ND; i++) {
        y1[i] = arg[i] + u[5][i];
        const double sc = m->o->atol[i] + m->o->rtol * fmax(fabs(y0[i]), fabs(y1[i]));
        e += (u[5][i] / sc) * (u[5][i] / sc);
    }
    *err = sqrt(e / ND);
    return 0;
}

/* Scaled RMS norm used by the starting-step estimate. */
static double rms_scaled(const orc_model *m, const double *v, const double *y)
{
    double e = 0.0;
    for (int i = 0; i < ND; i++) {
        const double sc = m->o->atol[i] + m->o->rtol * fabs(y[i]);
        e += (v[i] / sc) * (v[i] / sc);
    }
    return sqrt(e / ND);
}

/* Starting step size (Hairer, Norsett & Wanner, Solving ODEs I, sec. II.4),
 * order 4. */
static double initial_step(orc_model *m, const double *y0, double dt)
{
    double f0[ND], y1[ND], f1[ND], d[ND];
    if (rhs_real(m, y0, f0)) return dt;
    const double d0 = rms_scaled(m, y0, y0), d1 = rms_scaled(m, f0, y0);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > dt) h0 = dt;
    for (int i = 0; i < ND; i++) y1[i] = y0[i] + h0 * f0[i];
    if (rhs_real(m, y1, f1)) return h0;
    for (int i = 0; i < ND; i++) d[i] = f1[i] - f0[i];
    const double d2 = rms_scaled(m, d, y0) / h0;
    const double dm = d1 > d2 ? d1 : d2;
    double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 0.2);
    double h = 100.0 * h0 < h1 ? 100.0 * h0 : h1;
    return h < dt ? h : dt;
}

/* ------------------------------------------------------------------------ */
/* One coupling interval for one particle.                                  */
/* ------------------------------------------------------------------------ */
enum { ORC_OK = 0, ORC_ALGEBRAIC = 1, ORC_UNDERFLOW = 2, ORC_MAXSTEPS = 3,
       ORC_NONFINITE = 4, ORC_NEGATIVE = 0x80 };

static int finite_all(const double *v, int n)
{
    for (int i = 0; i < n; i++) if (!isfinite(v[i])) return 0;
    return 1;
}

/* x: 35-entry state, in place.  H_io / hlast_io: warm starts (<= 0: cold),
 * updated on success.  stats: accepted, rejected, algebraic Newton iterations.
 * kin: the kinetic factor of the particle's phase.  A failed particle keeps
 * its input state. */
static int advance(const orc_params *p, const orc_opts *o, double *x, double T, double D,
                   const double *s_in, double dt, double *H_io, double *hlast_io,
                   int *stats, double kin)
{
    orc_model m;
    m.p = p; m.o = o; m.c = phase_tconsts(p, T, kin); m.D = D;
    petersen(p, m.nu);
    for (int i = 0; i < NLIQ; i++) m.s_in[i] = s_in[i];
    m.H_guess = (H_io && *H_io > 0.0) ? *H_io : -1.0;
    m.Sh2_guess = x[S_H2];
    m.newton_iters = 0;
    stats[0] = stats[1] = stats[2] = 0;

    double y[ND], y1[ND];
    for (int k = 0; k < ND; k++) y[k] = x[DIFF[k]];
    if (!finite_all(y, ND) || !isfinite(T) || !isfinite(D) || !finite_all(s_in, NLIQ) ||
        !(T > 0.0) || !(dt > 0.0))
        return ORC_NONFINITE;

    /* the algebraic entries must be solvable at the start of the interval */
    {
        double f[ND];
        if (rhs_real(&m, y, f)) return ORC_ALGEBRAIC;
    }

    double h = (hlast_io && *hlast_io > 0.0) ? fmin(dt, *hlast_io) : initial_step(&m, y, dt);
    const double hmin = 1e-14 * dt;
    double t = 0.0;
    int reject_prev = 0, n = 0;
    for (;;) {
        if (n >= o->max_steps) return ORC_MAXSTEPS;
        if (h < hmin) return ORC_UNDERFLOW;
        double hs = h;
        int clip = 0;
        if (t + 1.01 * hs >= dt) { hs = dt - t; clip = 1; }
        double err = INFINITY;
        const int ok = rodas4_step(&m, y, hs, y1, &err) == 0 && finite_all(y1, ND) &&
                       isfinite(err);
        n++;
        double fac;
        if (!ok) fac = 0.2;
        else if (err == 0.0) fac = 5.0;
        else fac = fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.25)));
        double hnew = hs * fac;
        if (ok && err <= 1.0) {
            stats[0]++;
            memcpy(y, y1, sizeof(y));
            if (reject_prev && hnew > hs) hnew = hs;
            reject_prev = 0;
            if (clip) {
                if (hlast_io) *hlast_io = hnew > h ? hnew : h;
                break;
            }
            t += hs;
            h = hnew;
        } else {
            stats[1]++;
            reject_prev = 1;
            h = hnew;
        }
    }

    /* algebraic write-back at the end of the interval */
    cx yc[ND], xc[NX], H;
    for (int k = 0; k < ND; k++) yc[k] = y[k];
    if (algebraic(&m, yc, xc, &H)) return ORC_ALGEBRAIC;
    for (int i = 0; i < NX; i++) x[i] = creal(xc[i]);
    if (H_io) *H_io = creal(H);
    stats[2] = m.newton_iters;
    int st = ORC_OK;
    for (int k = 0; k < ND; k++) if (y[k] < 0.0) st |= ORC_NEGATIVE;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points.  State arrays are structure-of-arrays x[35][ld].  */
/* ------------------------------------------------------------------------ */
static void gather(const double *X, int64_t ld, int64_t i, double *x)
{
    for (int k = 0; k < NX; k++) x[k] = X[k * ld + i];
}
static void scatter(double *X, int64_t ld, int64_t i, const double *x)
{
    for (int k = 0; k < NX; k++) X[k * ld + i] = x[k];
}

typedef struct {
    const orc_params *p; const orc_opts *o;
    double *X; int64_t ld; const double *T; const double *D; const int32_t *fidx;
    const double *feed; double dt; double *H; double *hl; uint8_t *status;
    int32_t *stats; const double *kin; int64_t i0, i1;
} orc_job;

static void *run_chunk(void *arg)
{
    orc_job *j = (orc_job *)arg;
    for (int64_t i = j->i0; i < j->i1; i++) {
        double x[NX], x0[NX];
        gather(j->X, j->ld, i, x);
        memcpy(x0, x, sizeof(x));
        int st[3];
        double H = j->H ? j->H[i] : -1.0, hl = j->hl ? j->hl[i] : -1.0;
        const int s = advance(j->p, j->o, x, j->T[i], j->D[i],
                              j->feed + (int64_t)j->fidx[i] * NLIQ, j->dt, &H, &hl, st,
                              j->kin ? j->kin[i] : 1.0);
        if ((s & 0x7f) == ORC_OK) {
            scatter(j->X, j->ld, i, x);
            if (j->H) j->H[i] = H;
            if (j->hl) j->hl[i] = hl;
        } else {
            scatter(j->X, j->ld, i, x0);
        }
        j->status[i] = (uint8_t)s;
        if (j->stats)
            for (int k = 0; k < 3; k++) j->stats[k * j->ld + i] = st[k];
    }
    return NULL;
}

/* Advance particles 0..n-1 by dt.  feed: [n_feed][26] inflow concentrations,
 * fidx[i] selects particle i's row; D[i] its dilution rate (1/d); T[i] its
 * temperature (K).  H, hlast: warm starts (NULL or <= 0 entries: cold).
 * stats (nullable): [3][ld] accepted, rejected, Newton iterations.  kin
 * (nullable: all 1): kin[i] is the kinetic factor of particle i's phase. */
int orc_run(const orc_params *p, const orc_opts *o, double *X, int64_t ld,
            const double *T, const double *D, const int32_t *fidx, const double *feed,
            double dt, int64_t n, double *H, double *hlast, uint8_t *status,
            int32_t *stats, int nthreads, const double *kin)
{
    if (orc_check_params(p)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = (int)(n > 0 ? n : 1);
    pthread_t th[256];
    orc_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; t++) {
        orc_job *j = &jobs[t];
        j->p = p; j->o = o; j->X = X; j->ld = ld; j->T = T; j->D = D; j->fidx = fidx;
        j->feed = feed; j->dt = dt; j->H = H; j->hl = hlast; j->status = status;
        j->stats = stats; j->kin = kin;
        j->i0 = n * t / nthreads;
        j->i1 = n * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, run_chunk, &jobs[t]);
    run_chunk(&jobs[0]);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* f(y) for one particle.  x: 35-entry state (differential entries used, the
 * algebraic ones ignored except x[S_H2] as a starting guess).  Outputs: the
 * 28 derivatives in integration order, and the consistent 35-entry state
 * (algebraic entries solved) in x_alg, and S_H+ in *H.  Returns 0 / -1. */
int orc_rhs(const orc_params *p, const orc_opts *o, const double *x, double T, double D,
            const double *s_in, double *f, double *x_alg, double *H, double kin)
{
    orc_model m;
    m.p = p; m.o = o; m.c = phase_tconsts(p, T, kin); m.D = D;
    petersen(p, m.nu);
    for (int i = 0; i < NLIQ; i++) m.s_in[i] = s_in[i];
    m.H_guess = (H && *H > 0.0) ? *H : -1.0;
    m.Sh2_guess = x[S_H2];
    m.newton_iters = 0;
    cx y[ND], fc[ND], xc[NX], Hc;
    for (int k = 0; k < ND; k++) y[k] = x[DIFF[k]];
    if (rhs(&m, y, fc, &Hc)) return -1;
    for (int k = 0; k < ND; k++) f[k] = creal(fc[k]);
    if (x_alg) {
        if (algebraic(&m, y, xc, &Hc)) return -1;
        for (int i = 0; i < NX; i++) x_alg[i] = creal(xc[i]);
    }
    if (H) *H = creal(Hc);
    return 0;
}

/* Total Jacobian df/dy, 28x28 row-major, integration order. */
int orc_jacobian(const orc_params *p, const orc_opts *o, const double *x, double T,
                 double D, const double *s_in, double *J, double kin)
{
    orc_model m;
    m.p = p; m.o = o; m.c = phase_tconsts(p, T, kin); m.D = D;
    petersen(p, m.nu);
    for (int i = 0; i < NLIQ; i++) m.s_in[i] = s_in[i];
    m.H_guess = -1.0;
    m.Sh2_guess = x[S_H2];
    m.newton_iters = 0;
    double y[ND], f[ND];
    for (int k = 0; k < ND; k++) y[k] = x[DIFF[k]];
    if (rhs_real(&m, y, f)) return -1;
    return jacobian(&m, y, J);
}

/* Eq. 7 alone: S_H+ for the totals in x (35-entry layout). */
int orc_solve_ph(const orc_params *p, const orc_opts *o, const double *x, double T,
                 double guess, double *H)
{
    orc_tconst c = orc_tconsts(p, T);
    cx xc[NX], Hc;
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    if (solve_SH(p, o, &c, xc, guess, &Hc, NULL)) return -1;
    *H = creal(Hc);
    return 0;
}

/* Eq. 7 residual and eq. 8 residual at given S_H+ / S_h2 (for tests). */
double orc_charge_residual(const orc_params *p, const double *x, double T, double H)
{
    orc_tconst c = orc_tconsts(p, T);
    cx xc[NX];
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    return creal(charge_balance(p, &c, xc, H, NULL));
}

double orc_h2_residual(const orc_params *p, const double *x, double T, double H, double D,
                       double s_in_h2)
{
    orc_tconst c = orc_tconsts(p, T);
    double nu[NLIQ][NPROC];
    petersen(p, nu);
    cx xc[NX];
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    return creal(h2_balance(p, &c, xc, H, D, s_in_h2, nu, NULL));
}

/* Eq. 8 alone given S_H+. */
int orc_solve_h2(const orc_params *p, const orc_opts *o, const double *x, double T,
                 double H, double D, double s_in_h2, double *Sh2)
{
    orc_tconst c = orc_tconsts(p, T);
    double nu[NLIQ][NPROC];
    petersen(p, nu);
    cx xc[NX];
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    if (solve_Sh2(p, o, &c, xc, H, D, s_in_h2, nu, x[S_H2], NULL)) return -1;
    *Sh2 = creal(xc[S_H2]);
    return 0;
}

/* Rates for a full 35-entry state (S_h2 taken from x) and S_H+:
 * out[0..18] rho_j, out[19..21] transfers, out[22] gas flow per m3 liquid,
 * out[23..26] p_h2, p_ch4, p_co2, P_gas. */
void orc_rates(const orc_params *p, const double *x, double T, double H, double *out)
{
    orc_tconst c = orc_tconsts(p, T);
    cx xc[NX];
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    orc_rates_t r;
    rates(p, &c, xc, H, &r);
    for (int j = 0; j < NPROC; j++) out[j] = creal(r.rho[j]);
    for (int j = 0; j < 3; j++) out[NPROC + j] = creal(r.rhoT[j]);
    out[22] = creal(r.q_per_V);
    out[23] = creal(r.p_h2); out[24] = creal(r.p_ch4); out[25] = creal(r.p_co2);
    out[26] = creal(r.P_gas);
}

/* Gas flows of one particle with liquid volume V_liq (m3): q_gas, and the
 * h2, ch4, co2 shares q_gas p_i / P_gas, all m3/d. */
void orc_gas_flux(const orc_params *p, const double *x, double T, double V_liq,
                  double *q4)
{
    orc_tconst c = orc_tconsts(p, T);
    cx xc[NX];
    for (int i = 0; i < NX; i++) xc[i] = x[i];
    orc_rates_t r;
    rates(p, &c, xc, 1e-7, &r); /* S_H+ does not enter the gas flow */
    const double q = V_liq * creal(r.q_per_V), P = creal(r.P_gas);
    q4[0] = q;
    q4[1] = q * creal(r.p_h2) / P;
    q4[2] = q * creal(r.p_ch4) / P;
    q4[3] = q * creal(r.p_co2) / P;
}

/* Fixed-step integrators, nsteps equal steps over dt: classical RK4 and
 * Rodas4 without step control (the accuracy pins), and the explicit Euler
 * update y <- y + h f(y) of the paper's fixed-step scheme (sec. 2.3: small
 * synchronised steps need no step-size control; sec. 4.3: Dt = 0.5 s as ten
 * internal steps), method 2.  Every evaluation of f solves eqs. 7 and 8 at
 * the current differential state.  A non-finite state after a step fails. */
int orc_fixed(const orc_params *p, const orc_opts *o, double *x, double T, double D,
              const double *s_in, double dt, int nsteps, int method, double kin)
{
    orc_model m;
    m.p = p; m.o = o; m.c = phase_tconsts(p, T, kin); m.D = D;
    petersen(p, m.nu);
    for (int i = 0; i < NLIQ; i++) m.s_in[i] = s_in[i];
    m.H_guess = -1.0;
    m.Sh2_guess = x[S_H2];
    m.newton_iters = 0;
    double y[ND], h = dt / nsteps;
    for (int k = 0; k < ND; k++) y[k] = x[DIFF[k]];
    for (int s = 0; s < nsteps; s++) {
        if (method == 2) {
            double f[ND];
            if (rhs_real(&m, y, f)) return -1;
            for (int i = 0; i < ND; i++) y[i] += h * f[i];
            if (!finite_all(y, ND)) return -1;
        } else if (method == 0) {
            double k1[ND], k2[ND], k3[ND], k4[ND], a[ND];
            if (rhs_real(&m, y, k1)) return -1;
            for (int i = 0; i < ND; i++) a[i] = y[i] + 0.5 * h * k1[i];
            if (rhs_real(&m, a, k2)) return -1;
            for (int i = 0; i < ND; i++) a[i] = y[i] + 0.5 * h * k2[i];
            if (rhs_real(&m, a, k3)) return -1;
            for (int i = 0; i < ND; i++) a[i] = y[i] + h * k3[i];
            if (rhs_real(&m, a, k4)) return -1;
            for (int i = 0; i < ND; i++)
                y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        } else {
            double y1[ND], err;
            if (rodas4_step(&m, y, h, y1, &err)) return -1;
            memcpy(y, y1, sizeof(y));
        }
    }
    cx yc[ND], xc[NX], H;
    for (int k = 0; k < ND; k++) yc[k] = y[k];
    if (algebraic(&m, yc, xc, &H)) return -1;
    for (int i = 0; i < NX; i++) x[i] = creal(xc[i]);
    return 0;
}

/* The fixed-step scheme over particles 0..n-1 of x[35][ld], in equal chunks
 * over nthreads threads (the paper's CPU parallelisation, sec. 4.3): each
 * particle advances by dt in nsteps steps of `method` (orc_fixed).  status[i]
 * is 0, or 1 where the integration failed (the particle keeps its input). */
typedef struct {
    const orc_params *p; const orc_opts *o;
    double *X; int64_t ld; const double *T; const double *D; const int32_t *fidx;
    const double *feed; double dt; int nsteps, method; uint8_t *status; const double *kin;
    int64_t i0, i1;
} orc_fixed_job;

static void *run_fixed_chunk(void *arg)
{
    orc_fixed_job *j = (orc_fixed_job *)arg;
    for (int64_t i = j->i0; i < j->i1; i++) {
        double x[NX];
        gather(j->X, j->ld, i, x);
        const int rc = orc_fixed(j->p, j->o, x, j->T[i], j->D[i],
                                 j->feed + (int64_t)j->fidx[i] * NLIQ, j->dt, j->nsteps,
                                 j->method, j->kin ? j->kin[i] : 1.0);
        if (rc == 0) scatter(j->X, j->ld, i, x);
        j->status[i] = rc == 0 ? 0 : 1;
    }
    return NULL;
}

int orc_run_fixed(const orc_params *p, const orc_opts *o, double *X, int64_t ld,
                  const double *T, const double *D, const int32_t *fidx, const double *feed,
                  double dt, int nsteps, int method, int64_t n, uint8_t *status, int nthreads,
                  const double *kin)
{
    if (orc_check_params(p) || nsteps < 1) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = (int)(n > 0 ? n : 1);
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    orc_fixed_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        orc_fixed_job *j = &jobs[t];
        j->p = p; j->o = o; j->X = X; j->ld = ld; j->T = T; j->D = D; j->fidx = fidx;
        j->feed = feed; j->dt = dt; j->nsteps = nsteps; j->method = method;
        j->status = status; j->kin = kin;
        j->i0 = n * t / nthreads;
        j->i1 = n * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, run_fixed_chunk, &jobs[t]);
    run_fixed_chunk(&jobs[0]);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}
