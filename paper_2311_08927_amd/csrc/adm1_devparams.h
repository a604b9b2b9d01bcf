// Device-side parameter block of the ADM1 reaction step.
//
// Built once on the host by adm1_init from the named parameters (the
// standard ADM1 set; section 2.2) and passed to every kernel by value, so it
// lives in the kernel-argument segment and is read through scalar loads.
// Stoichiometric coefficients are evaluated on the host from the model
// description's expressions (e.g. (1 - Y_su) f_bu_su); the inorganic-carbon
// and -nitrogen rows of the Petersen matrix are the closures
// nuIC_j = -sum_i C_i nu_ij and nuIN_j = -sum_i N_i nu_ij.
#pragma once

#ifdef __cplusplus
namespace adm1 {
#endif

#define ADM1_NU_MAX 64  // room for the coefficient table of a model description

typedef struct DevParams {
    // kinetic constants at T_ref_kin (1/d, kg COD/m3, kmol/m3)
    double k_dis, k_hyd_ch, k_hyd_pr, k_hyd_li;
    double k_m_su, K_S_su, k_m_aa, K_S_aa, k_m_fa, K_S_fa, K_I_h2_fa;
    double k_m_c4, K_S_c4, K_I_h2_c4, k_m_pro, K_S_pro, K_I_h2_pro;
    double k_m_ac, K_S_ac, K_I_nh3, k_m_h2, K_S_h2;
    double k_dec[7];
    double K_S_IN, eps_c4;
    // pH inhibition (eqs. 3-4, Hill form in S_H+): I = 1 / (1 + (S_H/K)^n)
    double pH_K[3], pH_n[3];  // aa, ac, h2
    double pH_invK[3];        // 1 / pH_K
    int pH_nint[3];           // n when it is a small integer (1..4), else 0
    int pad0;
    // temperature dependence
    double Ea_R100, inv_T_ref_kin, inv_T_base, R;
    double K_w_base, dH_w_R100, K_a_co2_base, dH_a_co2_R100, K_a_IN_base, dH_a_IN_R100;
    double K_H_h2_base, dH_H_h2_R100, K_H_ch4_base, dH_H_ch4_R100, K_H_co2_base,
        dH_H_co2_R100;
    double p_h2o_base, p_h2o_coef;
    double K_a_va, K_a_bu, K_a_pro, K_a_ac;
    // gas phase: transfer, headspace, valve
    double kLa, kp, inv_vg, P_atm;
    double inv_P_atm, inv_K_I_nh3;
    // stoichiometry: the Petersen-matrix coefficients that are not +-1, in
    // the order of the generated table (adm1_stoich.inc, from the model
    // description), and the inorganic carbon / nitrogen closure rows
    double nu_v[ADM1_NU_MAX];
    double nuIC[19], nuIN[19];
    // integration control
    double rtol;
    double atol[28];
    double newton_tol;
    double newton_qtol;  // 0.1 sqrt(newton_tol): stop once a Newton correction is below it
    int max_steps, newton_maxit;
    double pivot_floor;  // growth guard of the static-order LU (0: off)
} DevParams;

#ifdef __cplusplus
}  // namespace adm1
#endif
