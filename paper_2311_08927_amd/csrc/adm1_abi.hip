// C ABI of the ADM1 step (declared in include/adm1.h): argument checking,
// parameter derivation, context scratch, and kernel dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "adm1.h"
#include "adm1_ctx.h"
#include "adm1_fixed.h"
#include "adm1_kernels.h"
#include "adm1_count.h"

using adm1::DevParams;

namespace {

constexpr int kGasBlocks = 1024;

// Scratch of adm1_step_particles_static, for callers that cannot allocate:
// the work-queue counter (word 0 of a 64-word area), the cost-order
// histogram, bucket cursors and list length, and the cost-ordered particle
// list of at most ADM1_STATIC_MAX_N particles.  Each device holds its own
// copy (4.2 MB) from module load to process end; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int64_t kStaticQueueWords = 64;
constexpr int64_t kStaticWorkWords = 2 * adm1::kOrderBuckets + 64;
constexpr int64_t kStaticClearWords = kStaticQueueWords + kStaticWorkWords;
constexpr int64_t kStaticWords = kStaticClearWords + ADM1_STATIC_MAX_N;
static_assert(2 * adm1::kOrderBuckets + 1 <= kStaticWorkWords, "cost-order work area");
static __device__ __align__(256) int32_t scratch[kStaticWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once).
int static_scratch(int dev, int32_t** out)
{
    if (dev < 0 || dev >= kMaxDevices) return ADM1_E_NOMEM;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return e != hipSuccess ? (int)e : ADM1_E_NOMEM;
        }
        g_scratch_dev[dev] = (int32_t*)p;
    }
    *out = g_scratch_dev[dev];
    return ADM1_OK;
}

__global__ void k_clear_words(int32_t* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

#define ADM1_PARAM_FIELDS(X)                                                              \
    X(f_sI_xc) X(f_xI_xc) X(f_ch_xc) X(f_pr_xc) X(f_li_xc) X(N_xc) X(N_I) X(N_aa) X(N_bac) \
    X(C_xc) X(C_sI) X(C_ch) X(C_pr) X(C_li) X(C_xI) X(C_su) X(C_aa) X(C_fa) X(C_va)      \
    X(C_bu) X(C_pro) X(C_ac) X(C_bac) X(C_ch4) X(f_fa_li) X(f_h2_su) X(f_bu_su)          \
    X(f_pro_su) X(f_ac_su) X(f_h2_aa) X(f_va_aa) X(f_bu_aa) X(f_pro_aa) X(f_ac_aa)       \
    X(f_ac_fa) X(f_h2_fa) X(f_pro_va) X(f_ac_va) X(f_h2_va) X(f_ac_bu) X(f_h2_bu)        \
    X(f_ac_pro) X(f_h2_pro) X(Y_su) X(Y_aa) X(Y_fa) X(Y_c4) X(Y_pro) X(Y_ac) X(Y_h2)     \
    X(k_dis) X(k_hyd_ch) X(k_hyd_pr) X(k_hyd_li) X(k_m_su) X(K_S_su) X(k_m_aa)          \
    X(K_S_aa) X(k_m_fa) X(K_S_fa) X(K_I_h2_fa) X(k_m_c4) X(K_S_c4) X(K_I_h2_c4)          \
    X(k_m_pro) X(K_S_pro) X(K_I_h2_pro) X(k_m_ac) X(K_S_ac) X(K_I_nh3) X(k_m_h2)        \
    X(K_S_h2) X(k_dec_su) X(k_dec_aa) X(k_dec_fa) X(k_dec_c4) X(k_dec_pro) X(k_dec_ac)  \
    X(k_dec_h2) X(K_S_IN) X(pH_UL_aa) X(pH_LL_aa) X(pH_UL_ac) X(pH_LL_ac) X(pH_UL_h2)  \
    X(pH_LL_h2) X(eps_c4) X(E_a) X(T_ref_kin) X(R) X(T_base) X(K_w_base) X(dH_w)        \
    X(K_a_va) X(K_a_bu) X(K_a_pro) X(K_a_ac) X(K_a_co2_base) X(dH_a_co2) X(K_a_IN_base) \
    X(dH_a_IN) X(K_H_h2_base) X(dH_H_h2) X(K_H_ch4_base) X(dH_H_ch4) X(K_H_co2_base)    \
    X(dH_H_co2) X(p_h2o_base) X(p_h2o_coef) X(k_L_a) X(k_p_per_V_liq) X(V_gas_per_V_liq) \
    X(P_atm)

const char kParamNames[] =
#define ADM1_NAME(n) #n ","
    ADM1_PARAM_FIELDS(ADM1_NAME)
#undef ADM1_NAME
    ;

// every field of adm1_params is listed once, in order
#define ADM1_COUNT(n) +1
static_assert(ADM1_FAIL_SLOTS == adm1::kFailSlots, "outcome counter slots");
// per-block partial outcome counts of the last step call
constexpr int kFailWords = adm1::kCountBlocks * adm1::kFailSlots;
static_assert(sizeof(adm1_params) == sizeof(double) * (0 ADM1_PARAM_FIELDS(ADM1_COUNT)),
              "adm1_params field list out of sync");
#undef ADM1_COUNT

enum E {
    eSsu, eSaa, eSfa, eSva, eSbu, eSpro, eSac, eSh2, eSch4, eSIC, eSIN, eSI, eXxc, eXch,
    eXpr, eXli, eXsu, eXaa, eXfa, eXc4, eXpro, eXac, eXh2, eXI, eScat, eSan, eNLIQ
};

#include <adm1_stoich.inc>
static_assert(ADM1_NU_COUNT <= ADM1_NU_MAX, "coefficient table of the model description");

// Petersen matrix of eq. 2 (organic entries; the inorganic C and N rows are
// derived as closures) from the named parameters, as the model description
// states it (generated).
void petersen(const adm1_params& p, double nu[eNLIQ][19])
{
    std::memset(nu, 0, sizeof(double) * eNLIQ * 19);
    ADM1_PETERSEN_FILL(p, nu);
}

int derive(const adm1_params& p, DevParams& d)
{
    std::memset(&d, 0, sizeof(d));
    // positivity of the constants that divide or set scales
    const double pos[] = {p.K_S_su, p.K_S_aa, p.K_S_fa, p.K_S_c4, p.K_S_pro, p.K_S_ac,
                          p.K_S_h2, p.K_I_h2_fa, p.K_I_h2_c4, p.K_I_h2_pro, p.K_I_nh3,
                          p.K_S_IN, p.eps_c4, p.R, p.T_base, p.T_ref_kin, p.K_w_base,
                          p.K_a_va, p.K_a_bu, p.K_a_pro, p.K_a_ac, p.K_a_co2_base,
                          p.K_a_IN_base, p.K_H_h2_base, p.K_H_ch4_base, p.K_H_co2_base,
                          p.V_gas_per_V_liq, p.P_atm, p.k_L_a};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v)) return ADM1_E_PARAMS;
    const double nonneg[] = {p.k_dis, p.k_hyd_ch, p.k_hyd_pr, p.k_hyd_li, p.k_m_su, p.k_m_aa,
                             p.k_m_fa, p.k_m_c4, p.k_m_pro, p.k_m_ac, p.k_m_h2, p.k_dec_su,
                             p.k_dec_aa, p.k_dec_fa, p.k_dec_c4, p.k_dec_pro, p.k_dec_ac,
                             p.k_dec_h2, p.k_p_per_V_liq, p.p_h2o_base};
    for (double v : nonneg)
        if (!(v >= 0.0) || !std::isfinite(v)) return ADM1_E_PARAMS;
    const double ll[3] = {p.pH_LL_aa, p.pH_LL_ac, p.pH_LL_h2};
    const double ul[3] = {p.pH_UL_aa, p.pH_UL_ac, p.pH_UL_h2};
    for (int k = 0; k < 3; ++k) {
        if (!(ul[k] > ll[k])) return ADM1_E_PARAMS;
        d.pH_n[k] = 3.0 / (ul[k] - ll[k]);
        d.pH_K[k] = std::pow(10.0, -0.5 * (ll[k] + ul[k]));
        d.pH_invK[k] = 1.0 / d.pH_K[k];
        const double r = std::nearbyint(d.pH_n[k]);
        // the kernels take the Hill power by multiplication: exponents 1..4
        if (!(std::fabs(d.pH_n[k] - r) < 1e-12 && r >= 1 && r <= 4)) return ADM1_E_PARAMS;
        d.pH_nint[k] = (int)r;
    }

    double nu[eNLIQ][19];
    petersen(p, nu);
    // COD continuity of every process over the COD-bearing entries
    const int cod[] = {eSsu, eSaa, eSfa, eSva, eSbu, eSpro, eSac, eSh2, eSch4, eSI, eXxc,
                       eXch, eXpr, eXli, eXsu, eXaa, eXfa, eXc4, eXpro, eXac, eXh2, eXI};
    for (int j = 0; j < 19; ++j) {
        double s = 0.0, a = 0.0;
        for (int i : cod) { s += nu[i][j]; a += std::fabs(nu[i][j]); }
        if (std::fabs(s) > 1e-12 * (a > 1.0 ? a : 1.0)) return ADM1_E_PARAMS;
    }
    // carbon and nitrogen contents; closures
    double C[eNLIQ] = {0}, N[eNLIQ] = {0};
    ADM1_CONTENTS(p, C, N);
    for (int j = 0; j < 19; ++j) {
        double sc = 0.0, sn = 0.0;
        for (int i = 0; i < eNLIQ; ++i) { sc += C[i] * nu[i][j]; sn += N[i] * nu[i][j]; }
        d.nuIC[j] = -sc;
        d.nuIN[j] = -sn;
    }

    d.k_dis = p.k_dis; d.k_hyd_ch = p.k_hyd_ch; d.k_hyd_pr = p.k_hyd_pr;
    d.k_hyd_li = p.k_hyd_li;
    d.k_m_su = p.k_m_su; d.K_S_su = p.K_S_su; d.k_m_aa = p.k_m_aa; d.K_S_aa = p.K_S_aa;
    d.k_m_fa = p.k_m_fa; d.K_S_fa = p.K_S_fa; d.K_I_h2_fa = p.K_I_h2_fa;
    d.k_m_c4 = p.k_m_c4; d.K_S_c4 = p.K_S_c4; d.K_I_h2_c4 = p.K_I_h2_c4;
    d.k_m_pro = p.k_m_pro; d.K_S_pro = p.K_S_pro; d.K_I_h2_pro = p.K_I_h2_pro;
    d.k_m_ac = p.k_m_ac; d.K_S_ac = p.K_S_ac; d.K_I_nh3 = p.K_I_nh3;
    d.k_m_h2 = p.k_m_h2; d.K_S_h2 = p.K_S_h2;
    d.k_dec[0] = p.k_dec_su; d.k_dec[1] = p.k_dec_aa; d.k_dec[2] = p.k_dec_fa;
    d.k_dec[3] = p.k_dec_c4; d.k_dec[4] = p.k_dec_pro; d.k_dec[5] = p.k_dec_ac;
    d.k_dec[6] = p.k_dec_h2;
    d.K_S_IN = p.K_S_IN; d.eps_c4 = p.eps_c4;
    const double R100 = 100.0 * p.R;
    d.Ea_R100 = p.E_a / R100; d.inv_T_ref_kin = 1.0 / p.T_ref_kin;
    d.inv_T_base = 1.0 / p.T_base; d.R = p.R;
    d.K_w_base = p.K_w_base; d.dH_w_R100 = p.dH_w / R100;
    d.K_a_co2_base = p.K_a_co2_base; d.dH_a_co2_R100 = p.dH_a_co2 / R100;
    d.K_a_IN_base = p.K_a_IN_base; d.dH_a_IN_R100 = p.dH_a_IN / R100;
    d.K_H_h2_base = p.K_H_h2_base; d.dH_H_h2_R100 = p.dH_H_h2 / R100;
    d.K_H_ch4_base = p.K_H_ch4_base; d.dH_H_ch4_R100 = p.dH_H_ch4 / R100;
    d.K_H_co2_base = p.K_H_co2_base; d.dH_H_co2_R100 = p.dH_H_co2 / R100;
    d.p_h2o_base = p.p_h2o_base; d.p_h2o_coef = p.p_h2o_coef;
    d.K_a_va = p.K_a_va; d.K_a_bu = p.K_a_bu; d.K_a_pro = p.K_a_pro; d.K_a_ac = p.K_a_ac;
    d.kLa = p.k_L_a; d.kp = p.k_p_per_V_liq; d.inv_vg = 1.0 / p.V_gas_per_V_liq;
    d.P_atm = p.P_atm;
    d.inv_P_atm = 1.0 / p.P_atm;
    d.inv_K_I_nh3 = 1.0 / p.K_I_nh3;
    ADM1_NU_VALUES(nu, d);
    return ADM1_OK;
}

int apply_opts(const adm1_opts& o, DevParams& d)
{
    if (!(o.rtol > 0.0) || !std::isfinite(o.rtol) || o.max_steps <= 0 ||
        !(o.newton_tol > 0.0) || o.newton_maxit <= 0 ||
        (o.rate_precision != 0 && o.rate_precision != 1) || o.variant < -1 ||
        o.variant >= ADM1_VARIANT_COUNT || !(o.pivot_floor >= 0.0) ||
        !std::isfinite(o.pivot_floor))
        return ADM1_E_OPTS;
    for (int k = 0; k < 28; ++k)
        if (!(o.atol[k] > 0.0) || !std::isfinite(o.atol[k])) return ADM1_E_OPTS;
    d.rtol = o.rtol;
    for (int k = 0; k < 28; ++k) d.atol[k] = o.atol[k];
    d.newton_tol = o.newton_tol;
    d.newton_qtol = 0.1 * std::sqrt(o.newton_tol);
    d.max_steps = o.max_steps;
    d.newton_maxit = o.newton_maxit;
    d.pivot_floor = o.pivot_floor;
    return ADM1_OK;
}

}  // namespace

namespace adm1_abi {

bool is_device(const void* ptr)
{
    if (!ptr) return false;
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
           at.type == hipMemoryTypeUnified;
}

int check_layout(const adm1_ctx* ctx, int64_t ld, int64_t n)
{
    if (n < 0 || n > ctx->n_max || ld < n || ld <= 0 || ld % 64 != 0) return ADM1_E_SIZE;
    return ADM1_OK;
}

int check_feed(const adm1_feed* feed)
{
    if (!feed) return ADM1_E_NULL;
    if (!feed->D || !feed->idx || !feed->S_in) return ADM1_E_NULL;
    if (feed->n_feed < 1) return ADM1_E_FEED;
    if (!is_device(feed->D) || !is_device(feed->idx) || !is_device(feed->S_in))
        return ADM1_E_NOT_DEVICE;
    if (feed->phase && !is_device(feed->phase)) return ADM1_E_NOT_DEVICE;
    return ADM1_OK;
}

int check_feed_no_phase(const adm1_feed* feed)
{
    const int rc = check_feed(feed);
    if (rc) return rc;
    return feed->phase ? ADM1_E_FEED : ADM1_OK;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? ADM1_OK : (int)e; }

int finish_capture(hipStream_t s, int rc, adm1_graph* g, adm1_graph** out)
{
    hipError_t e = hipStreamEndCapture(s, &g->graph);
    if (rc == ADM1_OK && e != hipSuccess) rc = (int)e;
    if (rc == ADM1_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = (int)e;
    }
    if (rc != ADM1_OK) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return rc;
    }
    *out = g;
    return ADM1_OK;
}

}  // namespace adm1_abi

using namespace adm1_abi;

namespace {
// The phase table of a context: kin[0..n-1], then 1 for every other id.
int set_phase_table(adm1_ctx* c, const double* kin, int32_t n)
{
    double t[ADM1_MAX_PHASES];
    for (int k = 0; k < ADM1_MAX_PHASES; ++k) t[k] = k < n ? kin[k] : 1.0;
    if (hipMemcpy(c->d_phase_kin, t, sizeof(t), hipMemcpyHostToDevice) != hipSuccess)
        return (int)hipGetLastError();
    return ADM1_OK;
}
}  // namespace

extern "C" {

const char* adm1_param_names(void) { return kParamNames; }

const char* adm1_model_name(void) { return ADM1_MODEL_NAME; }

const char* adm1_strerror(int code)
{
    switch (code) {
    case ADM1_OK: return "ok";
    case ADM1_E_NULL: return "a required pointer is NULL";
    case ADM1_E_SIZE: return "bad size: need 0 <= n <= n_max, ld >= n, ld % 64 == 0";
    case ADM1_E_NOT_DEVICE: return "pointer is not device memory";
    case ADM1_E_PARAMS: return "parameter set fails COD continuity or a range check";
    case ADM1_E_OPTS: return "invalid integration options";
    case ADM1_E_FEED: return "invalid feed table";
    case ADM1_E_NOMEM: return "context scratch allocation failed";
    case ADM1_E_VARIANT: return "unknown step-kernel variant";
    case ADM1_E_DT: return "dt must be positive and finite";
    case ADM1_E_IO: return "snapshot file missing, unreadable, unwritable or malformed";
    case ADM1_E_STATIC: return "n exceeds ADM1_STATIC_MAX_N, the capacity of the static scratch";
    default: break;
    }
    if (code > 0) return hipGetErrorString((hipError_t)code);
    return "unknown error";
}

int adm1_init(const adm1_params* p, const adm1_opts* o, int64_t n_max, adm1_ctx** out)
{
    if (!p || !o || !out) return ADM1_E_NULL;
    if (n_max < 0) return ADM1_E_SIZE;
    adm1_ctx* c = new (std::nothrow) adm1_ctx;
    if (!c) return ADM1_E_NOMEM;
    std::memset(c, 0, sizeof(*c));
    int rc = derive(*p, c->dp);
    if (rc == ADM1_OK) rc = apply_opts(*o, c->dp);
    if (rc != ADM1_OK) { delete c; return rc; }
    c->opts = *o;
    c->raw = *p;
    c->n_max = n_max;
    c->tuned_variant = -1;
    c->tuned_blocks_per_cu = 0;
    c->order_mode = ADM1_ORDER_COST;
    const size_t order_work = (2 * adm1::kOrderBuckets + 1) * sizeof(int32_t);
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return ADM1_E_NOMEM;
    }
    if (hipMalloc(&c->d_queue, 64 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->d_partial, kGasBlocks * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_params, sizeof(DevParams)) != hipSuccess ||
        hipMemcpy(c->d_params, &c->dp, sizeof(DevParams), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(c->d_queue, 0, 64 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->d_order, (size_t)(n_max > 0 ? n_max : 1) * sizeof(int32_t)) !=
            hipSuccess ||
        hipMalloc(&c->d_order_work, order_work) != hipSuccess ||
        hipMemset(c->d_order_work, 0, order_work) != hipSuccess ||
        hipMalloc(&c->d_fail, kFailWords * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->d_fail, 0, kFailWords * sizeof(unsigned long long)) !=
            hipSuccess ||
        hipMalloc(&c->d_phase_kin, ADM1_MAX_PHASES * sizeof(double)) != hipSuccess ||
        set_phase_table(c, nullptr, 0) != ADM1_OK ||
        static_scratch(c->device, &c->static_scratch) != ADM1_OK) {
        (void)hipGetLastError();
        if (c->d_queue) (void)hipFree(c->d_queue);
        if (c->d_partial) (void)hipFree(c->d_partial);
        if (c->d_params) (void)hipFree(c->d_params);
        if (c->d_order) (void)hipFree(c->d_order);
        if (c->d_order_work) (void)hipFree(c->d_order_work);
        if (c->d_fail) (void)hipFree(c->d_fail);
        if (c->d_phase_kin) (void)hipFree(c->d_phase_kin);
        delete c;
        return ADM1_E_NOMEM;
    }
    *out = c;
    return ADM1_OK;
}

int adm1_set_opts(adm1_ctx* ctx, const adm1_opts* o)
{
    if (!ctx || !o) return ADM1_E_NULL;
    DevParams d = ctx->dp;
    const int rc = apply_opts(*o, d);
    if (rc != ADM1_OK) return rc;
    if (hipMemcpy(ctx->d_params, &d, sizeof(DevParams), hipMemcpyHostToDevice) != hipSuccess)
        return (int)hipGetLastError();
    ctx->dp = d;
    ctx->opts = *o;
    return ADM1_OK;
}

void adm1_destroy(adm1_ctx* ctx)
{
    if (!ctx) return;
    (void)hipFree(ctx->d_queue);
    (void)hipFree(ctx->d_partial);
    (void)hipFree(ctx->d_params);
    (void)hipFree(ctx->d_order);
    (void)hipFree(ctx->d_order_work);
    (void)hipFree(ctx->d_fail);
    (void)hipFree(ctx->d_phase_kin);
    delete ctx;
}

int adm1_set_phase_kinetics(adm1_ctx* ctx, const double* kin, int32_t n_phases)
{
    if (!ctx) return ADM1_E_NULL;
    if (n_phases < 0 || n_phases > ADM1_MAX_PHASES) return ADM1_E_OPTS;
    if (n_phases > 0 && !kin) return ADM1_E_NULL;
    for (int32_t k = 0; k < n_phases; ++k)
        if (!std::isfinite(kin[k]) || kin[k] < 0.0) return ADM1_E_OPTS;
    return set_phase_table(ctx, kin, n_phases);
}

namespace {

// Work buffers of one step call: the queue counter, the cost-order work area
// and the ordered particle list (context scratch, or the static array).
struct StepScratch {
    int32_t* queue;
    int32_t* order_work;
    int32_t* order;
};

int check_step(adm1_ctx* ctx, double* state, int64_t ld, const double* temp_K,
               const adm1_feed* feed, double dt_days, int64_t n, adm1_aux* aux,
               uint8_t* status, int32_t* nsteps)
{
    if (!ctx || !state || !temp_K || !status) return ADM1_E_NULL;
    int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    rc = check_feed(feed);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(status)) return ADM1_E_NOT_DEVICE;
    if (nsteps && !is_device(nsteps)) return ADM1_E_NOT_DEVICE;
    if (aux) {
        if ((aux->H && !is_device(aux->H)) || (aux->h_last && !is_device(aux->h_last)))
            return ADM1_E_NOT_DEVICE;
    }
    return ADM1_OK;
}

// The step's launches on validated arguments: cost order (sparse2 with warm
// starts), the step kernel, the outcome counters.
int step_dispatch(adm1_ctx* ctx, const StepScratch& w, double* state, int64_t ld,
                  const double* temp_K, const adm1_feed* feed, double dt_days, int64_t n,
                  adm1_aux* aux, uint8_t* status, int32_t* nsteps, hipStream_t s)
{
    if (n == 0) return hip_rc(adm1::launch_count_status(status, 0, ctx->d_fail, s));
    adm1::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.dt = dt_days;
    a.phase = feed->phase; a.phase_kin = ctx->d_phase_kin;
    a.H = aux ? aux->H : nullptr;
    a.hlast = aux ? aux->h_last : nullptr;
    a.status = status; a.nsteps = nsteps; a.queue = w.queue;
    a.pdev = ctx->d_params;
    a.service_batch = ctx->tuned_service_batch;
    int variant = ctx->opts.variant;
    if (variant < 0) variant = ctx->tuned_variant >= 0 ? ctx->tuned_variant : ADM1_VARIANT_SPARSE2;
    int rc = ADM1_OK;
    switch (variant) {
    case ADM1_VARIANT_DENSE1:
        rc = hip_rc(adm1::launch_step1(a, ctx->opts.rate_precision, 0, s));
        break;
    case ADM1_VARIANT_SPARSE1:
        rc = hip_rc(adm1::launch_step1(a, ctx->opts.rate_precision, 1, s));
        break;
    case ADM1_VARIANT_SPARSE1_LDS:
        rc = hip_rc(adm1::launch_step1(a, ctx->opts.rate_precision, 2, s));
        break;
    case ADM1_VARIANT_SPARSE2:
        // expensive particles first (predicted by the previous interval's
        // last step size) so that the queue's tail is made of cheap ones
        if (ctx->order_mode == ADM1_ORDER_COST && a.hlast && n <= INT32_MAX) {
            rc = hip_rc(adm1::launch_cost_order(a.hlast, nullptr, nullptr, n, dt_days,
                                                w.order_work, w.order, s));
            if (rc) return rc;
            a.index = w.order;
            a.index_count = w.order_work + 2 * adm1::kOrderBuckets;
            a.index_bound = n;
        }
        rc = hip_rc(adm1::launch_step_sparse2(a, ctx->opts.rate_precision,
                                              ctx->tuned_blocks_per_cu, s));
        break;
    default:
        return ADM1_E_VARIANT;
    }
    if (rc) return rc;
    return hip_rc(adm1::launch_count_status(status, n, ctx->d_fail, s));
}

}  // namespace

int adm1_step_particles(adm1_ctx* ctx, double* state, int64_t ld, const double* temp_K,
                        const adm1_feed* feed, double dt_days, int64_t n, adm1_aux* aux,
                        uint8_t* status, int32_t* nsteps, void* stream)
{
    const int rc = check_step(ctx, state, ld, temp_K, feed, dt_days, n, aux, status, nsteps);
    if (rc) return rc;
    const StepScratch w{ctx->d_queue, ctx->d_order_work, ctx->d_order};
    return step_dispatch(ctx, w, state, ld, temp_K, feed, dt_days, n, aux, status, nsteps,
                         (hipStream_t)stream);
}

int adm1_step_particles_static(adm1_ctx* ctx, double* state, int64_t ld, const double* temp_K,
                               const adm1_feed* feed, double dt_days, int64_t n, adm1_aux* aux,
                               uint8_t* status, int32_t* nsteps, void* stream)
{
    int rc = check_step(ctx, state, ld, temp_K, feed, dt_days, n, aux, status, nsteps);
    if (rc) return rc;
    if (n > ADM1_STATIC_MAX_N) return ADM1_E_STATIC;
    int32_t* base = ctx->static_scratch;
    if (!base) return ADM1_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the last call's contents: clear the counter and the
    // cost-order histogram, which the kernels expect to start at zero
    hipLaunchKernelGGL(k_clear_words, dim3(9), dim3(256), 0, s, base, kStaticClearWords);
    if ((rc = hip_rc(hipGetLastError()))) return rc;
    const StepScratch w{base, base + kStaticQueueWords, base + kStaticClearWords};
    return step_dispatch(ctx, w, state, ld, temp_K, feed, dt_days, n, aux, status, nsteps, s);
}

int adm1_step_fixed(adm1_ctx* ctx, double* state, int64_t ld, const double* temp_K,
                    const adm1_feed* feed, double dt_days, int32_t substeps, int32_t method,
                    int64_t n, double* H, uint8_t* status, int32_t* newton, void* stream)
{
    if (!ctx || !state || !temp_K || !status) return ADM1_E_NULL;
    int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    if (substeps < 1 || substeps > (1 << 20)) return ADM1_E_OPTS;
    if (method != ADM1_FIXED_EULER && method != ADM1_FIXED_RK4) return ADM1_E_OPTS;
    rc = check_feed(feed);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(status)) return ADM1_E_NOT_DEVICE;
    if ((H && !is_device(H)) || (newton && !is_device(newton))) return ADM1_E_NOT_DEVICE;
    if (n == 0) return hip_rc(adm1::launch_count_status(status, 0, ctx->d_fail, (hipStream_t)stream));
    adm1::FixedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.dt = dt_days; a.substeps = substeps;
    a.phase = feed->phase; a.phase_kin = ctx->d_phase_kin;
    a.method = method; a.H = H; a.status = status; a.newton = newton;
    rc = hip_rc(adm1::launch_fixed(a, ctx->opts.rate_precision, (hipStream_t)stream));
    if (rc) return rc;
    return hip_rc(adm1::launch_count_status(status, n, ctx->d_fail, (hipStream_t)stream));
}

int adm1_last_failures(adm1_ctx* ctx, int64_t* host_out, void* stream)
{
    if (!ctx || !host_out) return ADM1_E_NULL;
    unsigned long long c[kFailWords];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c, ctx->d_fail, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_rc(e);
    for (int k = 0; k < adm1::kFailSlots; ++k) {
        int64_t t = 0;
        for (int b = 0; b < adm1::kCountBlocks; ++b) t += (int64_t)c[b * adm1::kFailSlots + k];
        host_out[k] = t;
    }
    return ADM1_OK;
}

int adm1_solve_ph(adm1_ctx* ctx, const double* state, int64_t ld, const double* temp_K,
                  int64_t n, const double* H_guess, double* H_out, double* pH_out,
                  uint8_t* status, void* stream)
{
    if (!ctx || !state || !temp_K || !H_out) return ADM1_E_NULL;
    const int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(H_out)) return ADM1_E_NOT_DEVICE;
    if ((H_guess && !is_device(H_guess)) || (pH_out && !is_device(pH_out)) ||
        (status && !is_device(status)))
        return ADM1_E_NOT_DEVICE;
    adm1::PhArgs a;
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.guess = H_guess;
    a.H_out = H_out; a.pH_out = pH_out; a.status = status;
    return hip_rc(adm1::launch_solve_ph(a, (hipStream_t)stream));
}

int adm1_set_order(adm1_ctx* ctx, int32_t mode)
{
    if (!ctx) return ADM1_E_NULL;
    if (mode != ADM1_ORDER_INDEX && mode != ADM1_ORDER_COST) return ADM1_E_OPTS;
    ctx->order_mode = mode;
    return ADM1_OK;
}

int adm1_cost_order(adm1_ctx* ctx, const double* h_last, double dt_days, int64_t n,
                    int32_t* order, void* stream)
{
    if (!ctx || !h_last || !order) return ADM1_E_NULL;
    if (n < 0 || n > INT32_MAX) return ADM1_E_SIZE;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    if (!is_device(h_last) || !is_device(order)) return ADM1_E_NOT_DEVICE;
    return hip_rc(adm1::launch_cost_order(h_last, nullptr, nullptr, n, dt_days,
                                          ctx->d_order_work, order, (hipStream_t)stream));
}

int adm1_gas_flux(adm1_ctx* ctx, const double* state, int64_t ld, const double* temp_K,
                  const double* V_liq, int64_t n, double* q_gas, double* q_ch4,
                  double* totals, void* stream)
{
    if (!ctx || !state || !temp_K || !totals) return ADM1_E_NULL;
    const int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(totals))
        return ADM1_E_NOT_DEVICE;
    if ((V_liq && !is_device(V_liq)) || (q_gas && !is_device(q_gas)) ||
        (q_ch4 && !is_device(q_ch4)))
        return ADM1_E_NOT_DEVICE;
    adm1::GasArgs a;
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.V_liq = V_liq;
    a.q_gas = q_gas; a.q_ch4 = q_ch4; a.partial = ctx->d_partial;
    // fixed partition of the particles over the blocks: depends on n only
    int64_t chunk = (n + kGasBlocks - 1) / kGasBlocks;
    chunk = (chunk + 255) / 256 * 256;
    if (chunk < 256) chunk = 256;
    a.chunk = chunk;
    int nblocks = (int)((n + chunk - 1) / chunk);
    if (nblocks < 1) nblocks = 1;
    return hip_rc(adm1::launch_gasflux(a, nblocks, totals, (hipStream_t)stream));
}

int adm1_rhs(adm1_ctx* ctx, const double* state, int64_t ld, const double* temp_K,
             const adm1_feed* feed, int64_t n, double* dxdt, int64_t ld_out, double* H_out,
             int32_t rate_precision, uint8_t* status, void* stream)
{
    if (!ctx || !state || !temp_K || !dxdt) return ADM1_E_NULL;
    int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    if (ld_out < n) return ADM1_E_SIZE;
    if (rate_precision != 0 && rate_precision != 1) return ADM1_E_OPTS;
    rc = check_feed(feed);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(dxdt)) return ADM1_E_NOT_DEVICE;
    if ((H_out && !is_device(H_out)) || (status && !is_device(status)))
        return ADM1_E_NOT_DEVICE;
    adm1::RhsArgs a;
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.dxdt = dxdt; a.ld_out = ld_out; a.H_out = H_out;
    a.status = status;
    a.phase = feed->phase; a.phase_kin = ctx->d_phase_kin;
    return hip_rc(adm1::launch_rhs(a, rate_precision, (hipStream_t)stream));
}

int adm1_jacobian(adm1_ctx* ctx, const double* state, int64_t ld, const double* temp_K,
                  const adm1_feed* feed, int64_t n, double* J, uint8_t* status, void* stream)
{
    if (!ctx || !state || !temp_K || !J) return ADM1_E_NULL;
    int rc = check_layout(ctx, ld, n);
    if (rc) return rc;
    rc = check_feed(feed);
    if (rc) return rc;
    if (!is_device(state) || !is_device(temp_K) || !is_device(J)) return ADM1_E_NOT_DEVICE;
    if (status && !is_device(status)) return ADM1_E_NOT_DEVICE;
    adm1::RhsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.status = status;
    a.phase = feed->phase; a.phase_kin = ctx->d_phase_kin;
    return hip_rc(adm1::launch_jacobian(a, J, (hipStream_t)stream));
}

int adm1_set_launch(adm1_ctx* ctx, int32_t variant, int32_t blocks_per_cu)
{
    if (!ctx) return ADM1_E_NULL;
    if (variant < 0 || variant >= ADM1_VARIANT_COUNT) return ADM1_E_VARIANT;
    if (blocks_per_cu < 0 || blocks_per_cu > 4) return ADM1_E_OPTS;
    ctx->tuned_variant = variant;
    ctx->tuned_blocks_per_cu = blocks_per_cu;
    return ADM1_OK;
}


int adm1_set_service_batch(adm1_ctx* ctx, int32_t pairs)
{
    if (!ctx) return ADM1_E_NULL;
    if (pairs < 0 || pairs > 32) return ADM1_E_OPTS;
    ctx->tuned_service_batch = pairs;
    return ADM1_OK;
}

int adm1_graph_capture_step(adm1_ctx* ctx, double* state, int64_t ld, const double* temp_K,
                            const adm1_feed* feed, double dt_days, int64_t n, adm1_aux* aux,
                            uint8_t* status, int32_t* nsteps, const double* V_liq,
                            double* q_gas, double* q_ch4, double* totals, void* stream,
                            adm1_graph** out)
{
    if (!ctx || !out || !stream) return ADM1_E_NULL;
    hipStream_t s = (hipStream_t)stream;
    // validate before capturing, so a bad argument leaves no open capture
    const int rc0 = adm1_step_particles(ctx, state, ld, temp_K, feed, dt_days, 0, aux,
                                        status, nsteps, stream);
    if (rc0 != ADM1_OK) return rc0;
    adm1_graph* g = new (std::nothrow) adm1_graph;
    if (!g) return ADM1_E_NOMEM;
    g->graph = nullptr;
    g->exec = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) { delete g; return (int)e; }
    int rc = adm1_step_particles(ctx, state, ld, temp_K, feed, dt_days, n, aux, status,
                                 nsteps, stream);
    if (rc == ADM1_OK)
        rc = adm1_gas_flux(ctx, state, ld, temp_K, V_liq, n, q_gas, q_ch4, totals, stream);
    return finish_capture(s, rc, g, out);
}

int adm1_graph_launch(adm1_graph* g, void* stream)
{
    if (!g) return ADM1_E_NULL;
    return hip_rc(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

void adm1_graph_destroy(adm1_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
