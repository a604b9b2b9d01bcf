/*
 * adm1.h -- C ABI of the MI355X per-particle ADM1 reaction step.
 *
 * The problem (Kumar et al., "Introducing CHAD", arXiv 2311.08927, sec. 2.3):
 * N independent particles, each a CSTR with its own ADM1 state, temperature
 * and feed, are advanced over one synchronised coupling interval dt.  The
 * state obeys the mass balance of eq. 2 with the standard ADM1 rates
 * (sec. 2.2) and inhibition forms (eqs. 3-6); S_H+ and S_h2 are algebraic,
 * fixed by the charge balance (eq. 7) and the hydrogen balance (eq. 8).
 * Around that step: the paper's own fixed-step explicit scheme (sec. 4.3),
 * the coupling driver between intervals (advection, inlet feed mask,
 * diffusion between particles), binary particle snapshots, and a learned
 * surrogate of the step with an exact fallback.
 *
 * Conventions common to every call
 *   - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors) unless stated otherwise; the caller owns them.  The library
 *     owns only the context and its scratch buffers.
 *   - `state` is float64 structure-of-arrays [35][ld]: entry k of particle i
 *     is state[k*ld + i]; ld >= n and ld % 64 == 0.  Entries (units kg COD/m3
 *     unless noted): 0 S_su, 1 S_aa, 2 S_fa, 3 S_va, 4 S_bu, 5 S_pro, 6 S_ac,
 *     7 S_h2, 8 S_ch4, 9 S_IC (kmol C/m3), 10 S_IN (kmol N/m3), 11 S_I,
 *     12 X_xc, 13 X_ch, 14 X_pr, 15 X_li, 16 X_su, 17 X_aa, 18 X_fa, 19 X_c4,
 *     20 X_pro, 21 X_ac, 22 X_h2, 23 X_I, 24 S_cat (kmol/m3), 25 S_an
 *     (kmol/m3), 26 S_va-, 27 S_bu-, 28 S_pro-, 29 S_ac-, 30 S_hco3- (kmol/m3),
 *     31 S_nh3 (kmol/m3), 32 G_h2, 33 G_ch4, 34 G_co2 (kmol/m3).
 *     Entries 7 and 26..31 are algebraic: on input only entry 7 is read (as a
 *     starting guess for eq. 8); on output all seven hold the values
 *     consistent with the final differential entries.
 *   - Time in days, temperature in K, dilution rates in 1/d, flows in m3/d.
 *   - `stream` is a hipStream_t (NULL: the default stream).  Calls only
 *     enqueue work: they neither allocate nor synchronise, so they may be
 *     captured into a hipGraph.  Exceptions are marked "synchronous".
 *   - Return value: 0 on success; a negative ADM1_E* code for an invalid
 *     argument (nothing is enqueued); a positive value is a HIP error code
 *     from a launch.  adm1_strerror() names them.
 *   - Per-particle outcomes go to `status` (uint8 per particle):
 *       0 ok, 1 algebraic solve failed at the interval start, 2 step size
 *       underflow, 3 max_steps reached, 4 non-finite input; bit 0x80 set
 *       (with code 0) when a differential entry ended negative.
 *     A particle with a nonzero code keeps its input state and warm starts.
 */
#ifndef ADM1_H
#define ADM1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ADM1_OK = 0,
    ADM1_E_NULL = -1,        /* a required pointer is NULL */
    ADM1_E_SIZE = -2,        /* n < 0, n > n_max, ld < n or ld % 64 != 0 */
    ADM1_E_NOT_DEVICE = -3,  /* a pointer that must be device memory is not */
    ADM1_E_PARAMS = -4,      /* parameter set fails COD/C/N continuity or range */
    ADM1_E_OPTS = -5,        /* invalid integration options */
    ADM1_E_FEED = -6,        /* feed table invalid (n_feed < 1) */
    ADM1_E_NOMEM = -7,       /* context scratch allocation failed (adm1_init) */
    ADM1_E_VARIANT = -8,     /* unknown kernel variant */
    ADM1_E_DT = -9,          /* dt not positive and finite */
    ADM1_E_IO = -10,         /* snapshot file missing, unreadable, unwritable or malformed */
    ADM1_E_STATIC = -11      /* n above ADM1_STATIC_MAX_N (adm1_step_particles_static) */
};

/* Status codes written per particle. */
enum {
    ADM1_ST_OK = 0, ADM1_ST_ALGEBRAIC = 1, ADM1_ST_UNDERFLOW = 2, ADM1_ST_MAXSTEPS = 3,
    ADM1_ST_NONFINITE = 4, ADM1_ST_NEGATIVE = 0x80
};

/* ADM1 parameters (sec. 2.2; values of the standard ADM1 set).  Host struct.
 * Stoichiometric fractions f_*, yields Y_*, carbon contents C_* (kmol C per
 * kg COD) and nitrogen contents N_* (kmol N per kg COD); kinetic constants at
 * T_ref_kin (1/d, kg COD/m3); pH limits of the Hill inhibitions (eqs. 3-4);
 * van't Hoff base values at T_base with enthalpies dH_* (J/mol); the gas
 * phase: k_L_a (1/d), headspace valve k_p per m3 liquid (m3/(d bar m3)),
 * V_gas/V_liq, P_atm (bar).  E_a (J/mol) sets the Arrhenius factor
 * exp(E_a/(100 R) (1/T_ref_kin - 1/T)) on k_dis, k_hyd, k_m and k_dec.  The
 * field order is also returned by adm1_param_names(). */
typedef struct adm1_params {
    double f_sI_xc, f_xI_xc, f_ch_xc, f_pr_xc, f_li_xc;
    double N_xc, N_I, N_aa, N_bac;
    double C_xc, C_sI, C_ch, C_pr, C_li, C_xI, C_su, C_aa, C_fa, C_va, C_bu, C_pro, C_ac,
        C_bac, C_ch4;
    double f_fa_li, f_h2_su, f_bu_su, f_pro_su, f_ac_su;
    double f_h2_aa, f_va_aa, f_bu_aa, f_pro_aa, f_ac_aa;
    double f_ac_fa, f_h2_fa, f_pro_va, f_ac_va, f_h2_va, f_ac_bu, f_h2_bu, f_ac_pro, f_h2_pro;
    double Y_su, Y_aa, Y_fa, Y_c4, Y_pro, Y_ac, Y_h2;
    double k_dis, k_hyd_ch, k_hyd_pr, k_hyd_li;
    double k_m_su, K_S_su, k_m_aa, K_S_aa, k_m_fa, K_S_fa, K_I_h2_fa;
    double k_m_c4, K_S_c4, K_I_h2_c4, k_m_pro, K_S_pro, K_I_h2_pro;
    double k_m_ac, K_S_ac, K_I_nh3, k_m_h2, K_S_h2;
    double k_dec_su, k_dec_aa, k_dec_fa, k_dec_c4, k_dec_pro, k_dec_ac, k_dec_h2;
    double K_S_IN;
    double pH_UL_aa, pH_LL_aa, pH_UL_ac, pH_LL_ac, pH_UL_h2, pH_LL_h2;
    double eps_c4, E_a, T_ref_kin;
    double R, T_base, K_w_base, dH_w;
    double K_a_va, K_a_bu, K_a_pro, K_a_ac;
    double K_a_co2_base, dH_a_co2, K_a_IN_base, dH_a_IN;
    double K_H_h2_base, dH_H_h2, K_H_ch4_base, dH_H_ch4, K_H_co2_base, dH_H_co2;
    double p_h2o_base, p_h2o_coef;
    double k_L_a, k_p_per_V_liq, V_gas_per_V_liq, P_atm;
} adm1_params;

/* Integration options.  Host struct.
 *   rtol, atol[28]: error control of the adaptive Rosenbrock integrator
 *     (scaled RMS norm, sc_i = atol_i + rtol max(|y0_i|, |y1_i|)) over the 28
 *     differential entries in integration order (state entries 0-6, 8-25,
 *     32-34).
 *   max_steps: attempted steps per particle per call (> 0).
 *   newton_tol, newton_maxit: relative step tolerance and iteration cap of
 *     the eq. 7 / eq. 8 Newton solves.
 *   rate_precision: 0 rates and eq. 2 assembly in FP64; 1 in FP32 (the eq. 7
 *     and eq. 8 solves and the linear algebra stay FP64).
 *   variant: step-kernel layout; -1 lets the library choose (the choice set
 *     by adm1_set_launch, else ADM1_VARIANT_SPARSE2); otherwise an
 *     ADM1_VARIANT_* value.
 *   pivot_floor (>= 0, finite): growth guard of the static-order
 *     factorisations (every variant but ADM1_VARIANT_DENSE1, which pivots):
 *     an attempted step whose Newton matrix has a pivot smaller in magnitude
 *     than pivot_floor times that row's diagonal entry before elimination is
 *     rejected like a step whose error estimate fails (the step size shrinks,
 *     which makes the matrix more diagonally dominant); 0 turns the guard
 *     off. */
typedef struct adm1_opts {
    double rtol;
    double atol[28];
    int32_t max_steps;
    double newton_tol;
    int32_t newton_maxit;
    int32_t rate_precision;
    int32_t variant;
    double pivot_floor;
} adm1_opts;

enum {
    ADM1_VARIANT_DENSE1 = 0,  /* one lane per particle, dense bordered LU, pivoting */
    ADM1_VARIANT_SPARSE1 = 1, /* one lane per particle, static-order sparse LU */
    ADM1_VARIANT_SPARSE2 = 2, /* two lanes per particle, register-resident sparse LU */
    ADM1_VARIANT_SPARSE1_LDS = 3, /* one lane per particle, static-order sparse LU with the
                                     matrix in LDS (64 particles and 124 KB per compute unit) */
    ADM1_VARIANT_COUNT = 4
};

/* Per-particle inputs of the open-reactor balance (device pointers).  D[i]:
 * dilution rate q/V of particle i (1/d, 0 = closed particle); idx[i]: row of
 * S_in giving its inflow concentrations; S_in: float64 [n_feed][26], inflow
 * of state entries 0..25 (entry 7 is the S_h2 inflow of eq. 8).
 * phase (nullable): uint8 phase id of each particle (sec. 5, particles of
 * several kinds such as sediments or inert matter).  A phase scales every
 * biochemical rate of eq. 2 of its particles by the phase's kinetic factor
 * (adm1_set_phase_kinetics; 0 = inert, reactions off); dilution and the
 * liquid-gas transfers act in every phase.  NULL: every particle has
 * factor 1. */
typedef struct adm1_feed {
    const double *D;
    const int32_t *idx;
    const double *S_in;
    int64_t n_feed;
    const uint8_t *phase;
} adm1_feed;

/* Number of phase ids (the uint8 range). */
#define ADM1_MAX_PHASES 256

/* Warm starts carried from one coupling interval to the next (device
 * pointers, length >= n): H[i] = S_H+ (kmol/m3), h_last[i] = the step size
 * proposed at the end of the previous interval (d).  Entries <= 0 mean cold
 * start (S_H+ from 1e-7, the first step from the Hairer-Norsett-Wanner
 * starting-step estimate).  The step updates them for successful particles. */
typedef struct adm1_aux {
    double *H;
    double *h_last;
} adm1_aux;

typedef struct adm1_ctx adm1_ctx;

/* Create a context for up to n_max particles on the current HIP device.
 * Derives the stoichiometric closures (inorganic C and N rows of the Petersen
 * matrix of eq. 2) and checks COD continuity of every process; copies the
 * parameters into the context.  Allocates the context scratch (work-queue
 * counters and reduction buffers).  Synchronous.  *out is set on success.
 * ADM1_E_PARAMS also when a Hill exponent of eqs. 3-4, 3 / (pH_UL - pH_LL),
 * is not an integer from 1 to 4 (the standard set gives 2, 3 and 3): the
 * kernels take that power by multiplication. */
int adm1_init(const adm1_params *p, const adm1_opts *o, int64_t n_max, adm1_ctx **out);

/* Replace the integration options (host struct) of a context.  Synchronous. */
int adm1_set_opts(adm1_ctx *ctx, const adm1_opts *o);

/* Advance particles 0..n-1 by dt_days IN PLACE (the per-particle ADM1 step
 * over one coupling interval, sec. 2.3).  state: [35][ld]; temp_K: [n];
 * feed: see adm1_feed (host struct holding device pointers); aux: warm starts
 * (host struct of device pointers, nullable: cold start for every particle);
 * status: [n] uint8; nsteps (nullable): int32 [3][ld] = accepted steps,
 * rejected steps, algebraic Newton iterations of each particle. */
int adm1_step_particles(adm1_ctx *ctx, double *state, int64_t ld, const double *temp_K,
                        const adm1_feed *feed, double dt_days, int64_t n, adm1_aux *aux,
                        uint8_t *status, int32_t *nsteps, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): adm1_step_particles
 * with the kernels' work buffers (work-queue counter, cost-order histogram
 * and the ordered particle list) in a static device array of the library
 * instead of the context's scratch.  Same arguments, results and outcome
 * counters (adm1_last_failures) as adm1_step_particles; the call allocates
 * nothing.  Limit: n <= ADM1_STATIC_MAX_N particles, else ADM1_E_STATIC and
 * nothing is enqueued.  Each device holds one copy of the array (about
 * 4.2 MB) from the library's first use until the process ends; every call on
 * a device shares it and the call clears what must start at zero, so calls
 * that overlap on one device (concurrent streams, threads, contexts) race
 * and must be serialised by the caller. */
enum { ADM1_STATIC_MAX_N = 1048576 };
int adm1_step_particles_static(adm1_ctx *ctx, double *state, int64_t ld, const double *temp_K,
                               const adm1_feed *feed, double dt_days, int64_t n, adm1_aux *aux,
                               uint8_t *status, int32_t *nsteps, void *stream);

/* The paper's own fixed-step scheme (sec. 2.3: coupling steps small enough
 * that no step-size control is needed; sec. 4.3: Dt = 0.5 s in ten internal
 * steps of 0.05 s).  Advances particles 0..n-1 by dt_days IN PLACE in
 * `substeps` equal explicit steps (1..2^20): method ADM1_FIXED_EULER
 * (y <- y + h f(y)) or ADM1_FIXED_RK4 (classical fourth order); every
 * evaluation of f solves S_H+ and S_h2 from eqs. 7-8 at the current state,
 * warm-started from the previous roots, and the algebraic entries are
 * written back at the end.  The rates use opts.rate_precision.  state, ld,
 * temp_K, feed as in adm1_step_particles; H (nullable, [n]): S_H+ warm start
 * in (<= 0: cold), root out; status: [n] uint8, 0 ok, 1 an algebraic solve
 * failed, 2 a step produced a non-finite state (the step is too long for
 * the explicit scheme), 4 non-finite or invalid input, bit 0x80 a negative
 * differential entry; a failed particle keeps its input.  newton (nullable,
 * [n] int32): algebraic Newton iterations per particle.  Asynchronous on
 * `stream`; no allocation.  Invalid arguments: ADM1_E_NULL, ADM1_E_SIZE,
 * ADM1_E_DT (dt_days not positive and finite), ADM1_E_OPTS (substeps or
 * method out of range), ADM1_E_FEED, ADM1_E_NOT_DEVICE. */
enum { ADM1_FIXED_EULER = 0, ADM1_FIXED_RK4 = 1 };
int adm1_step_fixed(adm1_ctx *ctx, double *state, int64_t ld, const double *temp_K,
                    const adm1_feed *feed, double dt_days, int32_t substeps, int32_t method,
                    int64_t n, double *H, uint8_t *status, int32_t *newton, void *stream);

/* Diffusion between particles (the paper names it as the missing transport
 * term besides advection, sec. 2.3, and as its next step).  Operator (the
 * paper fixes none): the SPH diffusion form on equal particle volumes V_p,
 * dC_i/dt = 2 D V_p sum_{j != i, r_ij < 2h} (C_i - C_j) W'(r_ij)/r_ij with
 * the 3-D Wendland C2 kernel of support 2h, on the 13 soluble differential
 * entries (S_su..S_ac, S_ch4, S_IC, S_IN, S_I, S_cat, S_an); explicit Euler
 * substeps.  The algebraic entries are refreshed by the next reaction step.
 * Neighbours are found on a uniform grid of cells of edge h over the box
 * [lo, hi] (particles outside it are clamped into the edge cells, which
 * stays exact, only slower).  Stability of the explicit steps: the kernel
 * factor integrates to sum_j V_p |W'/r| ~ 3.5 / h^2 for evenly spread
 * particles, but randomly placed ones reach about twice that, so the
 * operator's rates reach ~28 D / h^2 (Gershgorin) and a substep must stay
 * below ~0.07 h^2 / D; use dt/substeps <= 0.05 h^2 / D (longer substeps make
 * the concentrations of clustered particles oscillate and grow).  The
 * caller chooses substeps. */
typedef struct adm1_diffusion {
    double h;     /* smoothing length (m) */
    double D;     /* diffusivity of the soluble entries (m2/d) */
    double V_p;   /* liquid volume of every particle (m3) */
    double lo[3]; /* box of the neighbour grid (m) */
    double hi[3];
} adm1_diffusion;

typedef struct adm1_grid adm1_grid;

/* Allocate a neighbour grid for up to n_max particles (cell arrays, the
 * particle order and copies in cell order: about 280 B per particle and 8 B
 * per cell).  Synchronous.  ADM1_E_OPTS if a parameter is not positive and finite or the
 * grid (cells of edge h over the box) would exceed 2^26 cells; ADM1_E_SIZE
 * for n_max outside 1..2^31-1. */
int adm1_grid_create(const adm1_diffusion *d, int64_t n_max, adm1_grid **out);
/* Free a grid.  Synchronous.  NULL is a no-op. */
void adm1_grid_destroy(adm1_grid *g);

/* Diffuse the soluble entries of particles 0..n-1 over dt_days in
 * `substeps` explicit steps, IN PLACE.  state: [35][ld] float64; pos:
 * float32 [3][ld] positions (m, the layout of adm1_advect); neighbours
 * (nullable, [n] int32): number of particles within 2h of each.  Sums run in
 * a fixed order (cells, then ascending particle index), so results repeat
 * bit for bit.  Asynchronous on `stream`, no allocation; calls that share a
 * grid must not overlap. */
int adm1_diffuse(adm1_grid *g, double *state, int64_t ld, const float *pos, int64_t n,
                 double dt_days, int32_t substeps, int32_t *neighbours, void *stream);

/* Binary particle snapshots: the particle data exchanged with the flow
 * solver every coupling step (sec. 2.3), which the paper moves as ASCII and
 * names a main bottleneck (sec. 4.3).  File layout (little endian): a 64-byte
 * header ("ADM1SNAP", uint32 version 1, uint32 field mask, uint64 n, float64
 * time in s, 32 zero bytes), then the rows of each present field in mask-bit
 * order: positions float32 [3][n] (m), velocities float32 [3][n] (m/s),
 * densities float32 [n] (kg/m3), states float64 [35][n].  All buffers are
 * HOST memory (pinned memory makes the following device copy fastest), laid
 * out like the device arrays: row r of a field starts at r * ld elements.
 * Rows move with positional reads / writes of 8 MB chunks on up to 8
 * threads.  Synchronous. */
enum { ADM1_SNAP_POS = 1, ADM1_SNAP_VEL = 2, ADM1_SNAP_RHO = 4, ADM1_SNAP_STATE = 8 };

/* Write particles 0..n-1 of the non-NULL fields to `path` (replaced).
 * ADM1_E_SIZE unless 0 <= n <= ld, ld >= 1; ADM1_E_IO on a failed open or
 * write. */
int adm1_snapshot_write(const char *path, int64_t n, int64_t ld, double time_s, const float *pos,
                        const float *vel, const float *rho, const double *state);

/* Particle count, field mask and time of a snapshot (each output nullable).
 * ADM1_E_IO if the file is missing or not a snapshot. */
int adm1_snapshot_info(const char *path, int64_t *n, uint32_t *fields, double *time_s);

/* Read the fields whose destinations are non-NULL; *n_out (nullable) gets
 * the particle count.  ADM1_E_IO if the file is missing, malformed, shorter
 * or longer than its header says, or lacks a requested field; ADM1_E_SIZE if
 * ld < n.  Nothing is guaranteed about the destinations after an error. */
int adm1_snapshot_read(const char *path, int64_t ld, float *pos, float *vel, float *rho,
                       double *state, int64_t *n_out);

/* Headspace gas flows (sec. 1: release of gaseous components) of particles
 * 0..n-1: q_gas = V_liq k_p max(0, P_gas - P_atm) P_gas / P_atm and
 * q_ch4 = q_gas p_ch4 / P_gas (m3/d), with P_gas the sum of the partial
 * pressures and the water vapour pressure.  V_liq: [n] liquid volume of each
 * particle (m3; NULL = 1 m3).  q_gas, q_ch4: [n] outputs (nullable).
 * totals: [4] device output (q_gas, q_h2, q_ch4, q_co2 summed over the
 * particles) reduced in a fixed order, so bit-identical run to run. */
int adm1_gas_flux(adm1_ctx *ctx, const double *state, int64_t ld, const double *temp_K,
                  const double *V_liq, int64_t n, double *q_gas, double *q_ch4,
                  double *totals, void *stream);

/* Right-hand side of eq. 2 (and the gas balances) for the 28 differential
 * entries, with S_H+ and S_h2 solved from eqs. 7-8 at the given state.
 * dxdt: float64 [28][ld_out] in integration order; H_out (nullable): [n]
 * S_H+; rate_precision as in adm1_opts.  Status (nullable) gets 1 where an
 * algebraic solve failed. */
int adm1_rhs(adm1_ctx *ctx, const double *state, int64_t ld, const double *temp_K,
             const adm1_feed *feed, int64_t n, double *dxdt, int64_t ld_out, double *H_out,
             int32_t rate_precision, uint8_t *status, void *stream);

/* Eq. 7 alone (sec. 2.2: the charge balance fixes S_H+ once the ion totals
 * are known; the ions S_va-, S_bu-, S_pro-, S_ac-, S_hco3- and S_nh3 are
 * the equilibrium fractions K_a/(K_a + S_H+) of their totals at the
 * particle's temperature).  Solves for S_H+ of particles 0..n-1 from the
 * totals in state (entries 3-6, 9, 10, 24, 25 are read) by the Newton
 * iteration of the step, to a relative change below sqrt(opts.newton_tol)/10.
 * H_guess (nullable, [n]): starting values (<= 0 or NULL: 1e-7 kmol/m3).
 * Outputs: H_out [n] S_H+ in kmol/m3; pH_out (nullable) [n] = -log10(S_H+);
 * status (nullable) [n]: 0 ok, 1 no convergence, 4 non-finite input or
 * T <= 0; the outputs of a failed particle are NaN.  Asynchronous on
 * `stream`; no allocation. */
int adm1_solve_ph(adm1_ctx *ctx, const double *state, int64_t ld, const double *temp_K,
                  int64_t n, const double *H_guess, double *H_out, double *pH_out,
                  uint8_t *status, void *stream);

/* Outcome counts of the last adm1_step_particles, adm1_step_fixed or
 * adm1_surrogate_step call on this context (also when replayed from a
 * captured graph), counted on the device from its status array after the
 * step: host_out[0] particles with a nonzero status code, host_out[1..4]
 * particles with code 1..4, host_out[5] particles with code 0 whose
 * negative-entry bit is set, host_out[6] particles counted (the call's n).
 * host_out is HOST memory of 7 int64.  Synchronous: waits for `stream`
 * (where the step was enqueued) and reads the counters. */
enum { ADM1_FAIL_SLOTS = 7 };
int adm1_last_failures(adm1_ctx *ctx, int64_t *host_out, void *stream);

/* Total Jacobian df/dy of the 28 differential entries (the algebraic
 * unknowns eliminated through eqs. 7-8): float64 [n][28][28] row-major, for
 * tests.  Status (nullable) as in adm1_rhs. */
int adm1_jacobian(adm1_ctx *ctx, const double *state, int64_t ld, const double *temp_K,
                  const adm1_feed *feed, int64_t n, double *J, uint8_t *status,
                  void *stream);

/* Launch configuration of the step kernel used when opts.variant is -1:
 * variant (an ADM1_VARIANT_* value) and, for ADM1_VARIANT_SPARSE2, resident
 * blocks (waves) per compute unit of the persistent grid (1..4; 0 = 4, one
 * per SIMD, the most that fit the kernel's 40 KB of LDS per wave).
 * Set by the autotuner after timing the candidates.  Synchronous. */
int adm1_set_launch(adm1_ctx *ctx, int32_t variant, int32_t blocks_per_cu);

/* Service batching of the persistent step kernel (ADM1_VARIANT_SPARSE2):
 * pairs whose particle finished its interval wait until `pairs` of the wave
 * are free (or none is active) and are then written back and restarted
 * together, a pass the whole wave takes part in (1..32; 0 = the default 4).
 * Results do not depend on it.  Set by the autotuner.  Synchronous;
 * ADM1_E_OPTS outside 0..32. */
int adm1_set_service_batch(adm1_ctx *ctx, int32_t pairs);

/* Order in which the persistent step kernel (ADM1_VARIANT_SPARSE2) takes
 * particles from its work queue.  The particles are independent (sec. 4.3,
 * where they are split into equal static chunks per thread) but their costs
 * differ several-fold, so the tail of an index-ordered queue leaves a few
 * expensive particles running on otherwise idle waves.
 *   ADM1_ORDER_INDEX: 0..n-1.
 *   ADM1_ORDER_COST (default): the permutation of adm1_cost_order on
 *     aux->h_last, i.e. expected step count dt / h_last, largest first, cold
 *     particles first of all.  Used when aux and aux->h_last are given, by
 *     adm1_step_particles and for the fallback list of adm1_surrogate_step.
 * A particle's result does not depend on the order.  Returns ADM1_E_OPTS for
 * another mode.  Synchronous (no device work). */
enum { ADM1_ORDER_INDEX = 0, ADM1_ORDER_COST = 1 };
int adm1_set_order(adm1_ctx *ctx, int32_t mode);

/* The permutation behind ADM1_ORDER_COST: order[0..n-1] (int32, device) lists
 * the particles 0..n-1 by non-increasing bucket
 *   b_i = min(floor(8 dt_days / h_last[i]), 1023),  b_i = 1023 where
 *   h_last[i] <= 0 or is NaN (cold start: no prediction),
 * ties in an unspecified order (a counting sort).  h_last: [n] device.
 * Uses the context's histogram scratch: calls on one context must not
 * overlap (the step kernel's work queue has the same restriction).
 * Asynchronous on `stream`; n <= 2^31 - 1. */
int adm1_cost_order(adm1_ctx *ctx, const double *h_last, double dt_days, int64_t n,
                    int32_t *order, void *stream);

/* A coupling step captured as a HIP graph: adm1_step_particles followed by
 * adm1_gas_flux with fixed arguments (sec. 2.3: one synchronised coupling
 * interval).  Capture records kernel launches only (no memset nodes);
 * replays read the arrays' current contents, so the caller may update
 * state, feed and temperatures between replays.  `stream` (a hipStream_t,
 * not NULL) is used for capture and is left idle.  Synchronous. */
typedef struct adm1_graph adm1_graph;
int adm1_graph_capture_step(adm1_ctx *ctx, double *state, int64_t ld, const double *temp_K,
                            const adm1_feed *feed, double dt_days, int64_t n, adm1_aux *aux,
                            uint8_t *status, int32_t *nsteps, const double *V_liq,
                            double *q_gas, double *q_ch4, double *totals, void *stream,
                            adm1_graph **out);
/* Enqueue one replay of the captured step on `stream`. */
int adm1_graph_launch(adm1_graph *g, void *stream);
/* Free a captured graph.  Synchronous.  NULL is a no-op. */
void adm1_graph_destroy(adm1_graph *g);

/* ------------------------------------------------------------------------
 * Coupling driver (sec. 2.3): between coupling steps each AD particle moves
 * with its fluid particle, and particles in the inlet region receive feed.
 * The SPH flow field of the paper is replaced by a smooth analytic field in
 * a cylindrical tank: solid-body rotation omega (rad/s) plus axisymmetric
 * Stokes stream-function modes psi = sum_k a[k] r^2 (R^2 - r^2) sin(k pi z/H),
 * k = 1..nmodes (divergence free, tangent to all walls).
 * ------------------------------------------------------------------------ */
#define ADM1_FLOW_MODES 8
typedef struct adm1_flow {
    double omega;              /* rad/s */
    double R, H;               /* tank radius and height, m */
    double a[ADM1_FLOW_MODES]; /* stream-function amplitudes, 1/(m s) */
    int32_t nmodes;
} adm1_flow;

/* Move particles 0..n-1 for dt_seconds in `substeps` equal substeps: a
 * classical RK4 step of the meridional (axisymmetric) modes, then the turn
 * by omega h (the two commute), done as three area-preserving shears; a
 * particle that crosses a boundary by rounding is reflected back inside.
 * Positions are advanced in FP64 over all substeps and rounded to FP32 once
 * (in FP32, increments near the axial stagnation points round away and
 * particles collapse onto the axis).  pos: float32 [3][ld] device array
 * (x, y, z in m), in place. */
int adm1_advect(float *pos, int64_t ld, int64_t n, const adm1_flow *flow, double dt_seconds,
                int32_t substeps, void *stream);

/* Feed mask at the start of an interval: particles with z >= z_min and
 * x^2 + y^2 <= r_max^2 get D = D_zone (1/d) and feed row fidx_zone, the
 * others D = 0 and row fidx_out (closed particles).  D: float64 [n],
 * fidx: int32 [n], flag (nullable): uint8 [n] membership; device arrays. */
int adm1_feed_mask(const float *pos, int64_t ld, int64_t n, double z_min, double r_max,
                   double D_zone, int32_t fidx_zone, int32_t fidx_out, double *D,
                   int32_t *fidx, uint8_t *flag, void *stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the particle step.  The paper (sec. 2.2) keeps the
 * stiff acid-base and hydrogen dynamics algebraic (eqs. 7-8) because they
 * cripple explicit integration; here an MLP proposes the whole state after
 * one interval, an FP64 gate built on those same balances accepts or rejects
 * each proposal, and rejected particles are integrated exactly.
 *
 * Network 38 -> 256 -> 256 -> 256 -> 256 -> 35, GELU (erf form) after the
 * four hidden layers.  Input features (FP32, standardised, rounded to BF16,
 * row of 64 with columns 38..63 zero): log(max(x_k, floor_k)) for the 35
 * state entries, T (K), log(dt) and the feed flag (1 when D > 0).  Output:
 * the standardised increments of log(max(x_k, floor_k)) over the interval
 * (FP32, row of 48, columns 35..47 unused).  Weights BF16, accumulation and
 * outputs FP32; training keeps FP32 master weights and Adam moments
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error.
 *
 * Parameter vectors exchanged with the host (float32, ADM1_MLP_PARAMS
 * entries) hold, layer by layer, W ([in][out], row-major) then b ([out]).
 * ------------------------------------------------------------------------ */
#define ADM1_MLP_IN 38
#define ADM1_MLP_HIDDEN 256
#define ADM1_MLP_OUT 35
#define ADM1_MLP_PARAMS 216355
#define ADM1_MLP_FEAT_LD 64  /* BF16 elements per feature row */
#define ADM1_MLP_OUT_LD 48   /* FP32 elements per output row */

typedef struct adm1_mlp_norm {
    float in_mean[ADM1_MLP_IN], in_sd[ADM1_MLP_IN];
    float out_mean[ADM1_MLP_OUT], out_sd[ADM1_MLP_OUT];
    double floor[ADM1_MLP_OUT]; /* floor_k > 0, per state entry */
} adm1_mlp_norm;

/* Acceptance thresholds of a proposal x^ = max(x, floor) exp(delta); every
 * test is strict, so an all-zero gate sends every particle to the exact
 * integrator.
 *   max_dlog:    |delta_k| for every entry;
 *   tol_ion:     proposed ions and S_h2 against their eq. 7 / eq. 8 values at
 *                the proposal's totals, relative to max(|value|, 100 floor);
 *   tol_closure: COD (liquid and headspace) and nitrogen balances over the
 *                interval (eq. 2 summed with COD and N weights): the change
 *                of each total must lie within dt times the range its
 *                boundary flux (dilution exchange, gas outflow) can span
 *                when each factor of the flux moves monotonically between
 *                its end-point values; the distance outside, relative to
 *                the pre-step total, is compared. */
typedef struct adm1_gate {
    double max_dlog;
    double tol_ion;
    double tol_closure;
} adm1_gate;

typedef struct adm1_surrogate adm1_surrogate;

/* Surrogate on a context: buffers for inference over up to n_max particles
 * (n_max <= the context's) and training batches of up to batch_max rows.
 * Weights start at zero.  Synchronous. */
int adm1_surrogate_create(adm1_ctx *ctx, int64_t n_max, int64_t batch_max,
                          adm1_surrogate **out);

/* Load weights (host float32 [ADM1_MLP_PARAMS]) and normalisation (host
 * struct); resets the Adam moments.  Synchronous. */
int adm1_surrogate_set_weights(adm1_surrogate *s, const float *params,
                               const adm1_mlp_norm *norm);

/* Copy the FP32 master weights (nullable) and normalisation (nullable) to
 * the host.  Synchronous. */
int adm1_surrogate_get_weights(adm1_surrogate *s, float *params, adm1_mlp_norm *norm);

/* Copy the gradients of the last training step (host float32
 * [ADM1_MLP_PARAMS], same layout as the weights).  Synchronous. */
int adm1_surrogate_get_grads(adm1_surrogate *s, float *grads);

/* Network inputs of particles 0..n-1: X = BF16 [n][64] (uint16 bit patterns,
 * 16-byte aligned, else ADM1_E_SIZE).  D: [n] dilution rates (the feed flag
 * is D > 0). */
int adm1_surrogate_featurize(adm1_surrogate *s, const double *state, int64_t ld,
                             const double *temp_K, const double *D, double dt_days, int64_t n,
                             uint16_t *X, void *stream);

/* Training targets from a pair of states one interval apart: float32
 * [n][35] standardised increments of log(max(x, floor)). */
int adm1_surrogate_targets(adm1_surrogate *s, const double *x0, const double *x1, int64_t ld,
                           int64_t n, float *target, void *stream);

/* Network outputs Y = float32 [n][48] for inputs X = BF16 [n][64] (X
 * 16-byte aligned, else ADM1_E_SIZE). */
int adm1_surrogate_forward(adm1_surrogate *s, const uint16_t *X, int64_t n, float *Y,
                           void *stream);

/* The gate alone, on given network outputs Y ([n][48]): accepted particles
 * get the proposal with eq. 7 / eq. 8 values in entries 7 and 26..31,
 * status 0, nsteps 0 and (aux->H) the solved S_H+; rejected particles keep
 * their state and have their index appended to fb_idx ([n] int32), in no
 * particular order; *fb_count (device int32) is set to their number.
 * route (nullable): [n] uint8, 1 accepted / 0 rejected. */
int adm1_surrogate_gate(adm1_surrogate *s, double *state, int64_t ld, const double *temp_K,
                        const adm1_feed *feed, double dt_days, int64_t n, const float *Y,
                        const adm1_gate *gate, adm1_aux *aux, uint8_t *status,
                        int32_t *nsteps, uint8_t *route, int32_t *fb_idx, int32_t *fb_count,
                        void *stream);

/* One coupling step through the surrogate: featurize, forward, gate, then
 * the exact step (ADM1_VARIANT_SPARSE2 kernel) on the rejected particles
 * from their pre-step states.  Arguments as in adm1_step_particles and
 * adm1_surrogate_gate; fb_count (nullable, device int32) receives the number
 * of rejected particles.  n <= the surrogate's n_max.  The surrogate models
 * one phase: a feed with a phase array is ADM1_E_FEED here and in
 * adm1_surrogate_gate and adm1_surrogate_graph_capture_step. */
int adm1_surrogate_step(adm1_surrogate *s, double *state, int64_t ld, const double *temp_K,
                        const adm1_feed *feed, double dt_days, int64_t n,
                        const adm1_gate *gate, adm1_aux *aux, uint8_t *status,
                        int32_t *nsteps, uint8_t *route, int32_t *fb_count, void *stream);

/* The gated surrogate step followed by adm1_gas_flux, captured as a HIP graph
 * (launched and destroyed with adm1_graph_launch / adm1_graph_destroy).
 * Arguments as in adm1_surrogate_step and adm1_gas_flux; the capture records
 * kernel launches only (the fallback count is cleared by a kernel and read
 * by the fallback kernel from device memory).  `stream` (a hipStream_t, not
 * NULL) is used for capture and left idle.  Synchronous. */
int adm1_surrogate_graph_capture_step(adm1_surrogate *s, double *state, int64_t ld,
                                      const double *temp_K, const adm1_feed *feed,
                                      double dt_days, int64_t n, const adm1_gate *gate,
                                      adm1_aux *aux, uint8_t *status, int32_t *nsteps,
                                      uint8_t *route, int32_t *fb_count, const double *V_liq,
                                      double *q_gas, double *q_ch4, double *totals,
                                      void *stream, adm1_graph **out);

/* One training step on a batch of B rows: X BF16 [B][64], target float32
 * [B][35]; forward, mean-squared-error loss (written to *loss, device
 * float32, before the update), backward, Adam with learning rate lr at step
 * number `step` (>= 1, for the bias corrections). */
int adm1_surrogate_train_step(adm1_surrogate *s, const uint16_t *X, const float *target,
                              int64_t B, float lr, int32_t step, float *loss, void *stream);

/* Mean residual and mean squared residual of the network, per output
 * column: over rows 0..n-1 of X (BF16 features [n][ADM1_MLP_FEAT_LD],
 * device) and target (float32 [n][ADM1_MLP_OUT], device, standardised
 * units), mean_out[c] = mean(Y[r][c] - target[r][c]) and msq_out[c] =
 * mean((Y - target)^2) for c < ADM1_MLP_OUT (HOST memory of 35 float64
 * each); the forward pass runs `chunk` rows at a time.  Sums in FP64 in a
 * fixed order (bit-reproducible).  Allocates a chunk of outputs and the
 * partial sums for the call.  Synchronous. */
int adm1_surrogate_residual_stats(adm1_surrogate *s, const uint16_t *X, const float *target,
                                  int64_t n, int64_t chunk, double *mean_out, double *msq_out,
                                  void *stream);

/* Free the surrogate.  Synchronous.  NULL is a no-op. */
void adm1_surrogate_destroy(adm1_surrogate *s);

/* Comma-separated adm1_params field names in struct order (static string). */
const char *adm1_param_names(void);

/* Kinetic factors of the particle phases (sec. 5, multiple phases): kin is
 * HOST memory of n_phases (0..ADM1_MAX_PHASES) float64 factors, each finite
 * and >= 0; phase id k < n_phases gets kin[k], every other id 1 (the
 * factors a new context starts with).  ADM1_E_OPTS for a bad count or
 * factor (the table is then unchanged).  Synchronous.  Not supported by the
 * surrogate calls (a feed with phases is ADM1_E_FEED there). */
int adm1_set_phase_kinetics(adm1_ctx *ctx, const double *kin, int32_t n_phases);

/* ------------------------------------------------------------------------
 * Data handling of the surrogate's training driver, on the device.
 * ------------------------------------------------------------------------ */
/* dst row j = src row idx[j] for j < n_idx, rows of row_bytes bytes (a
 * multiple of 4; src and dst 4-byte aligned); src has n_src rows, and an
 * index outside [0, n_src) yields a zero row.  Device arrays; idx int32.
 * Asynchronous on `stream`. */
int adm1_gather_rows(const void *src, int64_t n_src, int64_t row_bytes, const int32_t *idx,
                     int64_t n_idx, void *dst, void *stream);

/* out[0..n-1] (int32, device) = a permutation of 0..n-1 determined by
 * `seed`: a four-round Feistel network on the smallest even bit width
 * covering n, restricted to [0, n) by cycle walking.  n <= 2^31 - 1.
 * Asynchronous on `stream`. */
int adm1_permutation(int64_t n, uint64_t seed, int32_t *out, void *stream);

/* Per-column mean and sample standard deviation (divisor n - 1) of the
 * first `cols` (<= 64) columns of a row-major device array of n >= 2 rows
 * and ld elements per row, float32 (bf16 = 0) or BF16 bit patterns
 * (bf16 = 1), summed in FP64 in a fixed order (two passes, the second about
 * the mean).  mean_out, sd_out: HOST memory of cols float64.  Allocates its
 * partial sums for the call.  Synchronous. */
int adm1_column_stats(const void *data, int32_t bf16, int64_t n, int32_t cols, int64_t ld,
                      double *mean_out, double *sd_out, void *stream);

/* Name of the model description this library was generated from (sec. 2.2,
 * eq. 2: the Petersen matrix as data; static string): "adm1" for the
 * standard matrix.  The matrix's sparsity is compiled into the kernels, so
 * each description is its own library. */
const char *adm1_model_name(void);

/* Human-readable name of an ADM1_E* or HIP error code (static string). */
const char *adm1_strerror(int code);

/* Free the context and its scratch.  Synchronous.  NULL is a no-op. */
void adm1_destroy(adm1_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* ADM1_H */
