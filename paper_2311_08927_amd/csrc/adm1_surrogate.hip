// Learned surrogate of the per-particle step (declared in include/adm1.h):
// the BF16 MLP proposes the state after one coupling interval, an FP64 gate
// accepts or rejects each proposal, and rejected particles are integrated by
// the FP64 Rosenbrock kernel from their pre-step state through an index list.
//
// Gate of a proposal x^ = max(x, floor) exp(delta), per particle, in FP64:
//   domain   every delta finite with |delta| < max_dlog;
//   eq. 7    S_H+ solved from the proposal's totals; the proposed ions must
//            agree with their equilibrium values at that S_H+ (relative to
//            max(|value|, 100 floor) < tol_ion);
//   eq. 8    S_h2 solved at that pH; the proposed S_h2 must agree likewise;
//   closure  the changes of COD (liquid + headspace) and nitrogen over the
//            interval must lie within dt times the range the boundary fluxes
//            (dilution exchange, gas outflow) can span when each of their
//            factors moves monotonically between its end-point values; the
//            distance outside, relative to the pre-step totals, must be
//            below tol_closure.
// On pass the algebraic entries are replaced by the solved values (the
// proposal's differential entries are kept); on failure the particle is
// left untouched and its index appended to the fallback list.  All
// comparisons are strict, so an all-zero gate rejects every proposal.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "adm1.h"
#include "adm1_ctx.h"
#include "adm1_kernels.h"
#include "adm1_mlp.h"
#include "adm1_model.h"

using namespace adm1_abi;

namespace adm1 {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct GateConsts {
    double cod_w[NX];    // COD weight of each state row (liquid, headspace)
    double n_w[NX];      // nitrogen content of each state row
    double cod_in_w[NLIQ];
    double n_in_w[NLIQ];
    double floor_[NX];
    float out_mean[kMlpOut], out_sd[kMlpOut];
    double max_dlog, tol_ion, tol_closure;
};

struct GateArgs {
    DevParams p;
    GateConsts g;
    double* state;
    int64_t ld, n;
    const double* T;
    const double* D;
    const int32_t* fidx;
    const double* S_in;
    int64_t n_feed;
    double dt;
    const float* Y;       // [n][48]
    double* H;            // nullable
    uint8_t* status;
    int32_t* nsteps;      // nullable
    uint8_t* route;       // nullable
    int32_t* fb_idx;
    int32_t* fb_count;
};

// Gas flow per unit liquid volume (the gas-flow law of the headspace).
__device__ __forceinline__ double qgas(const DevParams& p, const TConst& c, const double* x)
{
    const double P = x[32] * c.RT * (1.0 / 16.0) + x[33] * c.RT * (1.0 / 64.0) + x[34] * c.RT +
                     c.p_h2o;
    return P > p.P_atm ? p.kp * (P - p.P_atm) * P / p.P_atm : 0.0;
}

struct NullSink {
    __device__ void operator()(int, double) const {}
};

// Every loop has a fixed trip count and is unrolled, so the per-particle
// arrays live in registers (a loop with an early exit would put them in
// scratch memory); the network's output row is read as nine 16-byte loads.
__global__ void __launch_bounds__(256) k_gate(GateArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool pass = false;
    if (i < a.n) {
        const DevParams& p = a.p;
        const GateConsts& g = a.g;
        double x0[NX], xh[NX];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            x0[k] = a.state[k * a.ld + i];
            ok = ok && isfinite(x0[k]);
        }
        const double T = a.T[i], D = a.D[i];
        const int fi = a.fidx[i];
        ok = ok && isfinite(T) && T > 0.0 && isfinite(D) && fi >= 0 && fi < a.n_feed;
        float yv[36];
        {
            const f32x4* yrow = (const f32x4*)(a.Y + i * kMlpOutPad);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const f32x4 v = yrow[q];
#pragma unroll
                for (int t = 0; t < 4; ++t) yv[4 * q + t] = v[t];
            }
        }
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k) {
            const double d = (double)yv[k] * g.out_sd[k] + g.out_mean[k];
            ok = ok && isfinite(d) && fabs(d) < g.max_dlog;
            xh[k] = fmax(x0[k], g.floor_[k]) * exp(d);
        }
        if (ok) {
            const double* sin = a.S_in + (int64_t)fi * NLIQ;
            const TConst c = tconst(p, T);
            double y[NY];
#pragma unroll
            for (int k = 0; k < NY; ++k) y[k] = xh[state_row(k)];
            double H = a.H ? a.H[i] : -1.0;
            double Sh2 = xh[ROW_SH2];
            int iters = 0;
            ok = rhs_in<double>(p, c, y, D, FeedInflow{D, sin}, H, Sh2, NullSink{}, iters) == 0;
            if (ok) {
                double ion[7];
                ion[0] = Sh2;
                ion[1] = p.K_a_va * y[Sva] / (p.K_a_va + H);
                ion[2] = p.K_a_bu * y[Sbu] / (p.K_a_bu + H);
                ion[3] = p.K_a_pro * y[Spro] / (p.K_a_pro + H);
                ion[4] = p.K_a_ac * y[Sac] / (p.K_a_ac + H);
                ion[5] = c.K_a_co2 * y[SIC] / (c.K_a_co2 + H);
                ion[6] = c.K_a_IN * y[SIN] / (c.K_a_IN + H);
                double worst = 0.0;
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    const int row = k == 0 ? ROW_SH2 : 25 + k;
                    const double sc = fmax(fabs(ion[k]), 100.0 * g.floor_[row]);
                    worst = fmax(worst, fabs(xh[row] - ion[k]) / sc);
                }
                ok = worst < g.tol_ion;
                // closure of COD and nitrogen over the interval
                double cin = 0.0, nin = 0.0;
#pragma unroll
                for (int k = 0; k < NLIQ; ++k) {
                    cin += g.cod_in_w[k] * sin[k];
                    nin += g.n_in_w[k] * sin[k];
                }
                xh[ROW_SH2] = Sh2;
#pragma unroll
                for (int k = 0; k < 6; ++k) xh[26 + k] = ion[1 + k];
                double C0 = 0.0, C1 = 0.0, N0 = 0.0, N1 = 0.0, L0 = 0.0, L1 = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) {
                    C0 += g.cod_w[k] * x0[k];
                    C1 += g.cod_w[k] * xh[k];
                    N0 += g.n_w[k] * x0[k];
                    N1 += g.n_w[k] * xh[k];
                    if (k < NLIQ) {
                        L0 += g.cod_w[k] * x0[k];
                        L1 += g.cod_w[k] * xh[k];
                    }
                }
                // the boundary fluxes over the interval lie between the
                // products of their factors' end-point extremes when each
                // factor is monotone in time
                const double q0 = qgas(p, c, x0), q1 = qgas(p, c, xh);
                const double g0 = x0[32] + x0[33], g1 = xh[32] + xh[33];
                const double Fc_lo = D * (cin - fmax(L0, L1)) - fmax(q0, q1) * fmax(g0, g1);
                const double Fc_hi = D * (cin - fmin(L0, L1)) - fmin(q0, q1) * fmin(g0, g1);
                const double Fn_lo = D * (nin - fmax(N0, N1)), Fn_hi = D * (nin - fmin(N0, N1));
                const double dC = C1 - C0, dN = N1 - N0;
                const double rc =
                    fmax(0.0, fmax(a.dt * Fc_lo - dC, dC - a.dt * Fc_hi)) / fabs(C0);
                const double rn =
                    fmax(0.0, fmax(a.dt * Fn_lo - dN, dN - a.dt * Fn_hi)) / fabs(N0);
                ok = ok && rc < g.tol_closure && rn < g.tol_closure;
                if (ok) {
#pragma unroll
                    for (int k = 0; k < NX; ++k) a.state[k * a.ld + i] = xh[k];
                    if (a.H) a.H[i] = H;
                    a.status[i] = 0;
                    if (a.nsteps) {
                        a.nsteps[i] = 0;
                        a.nsteps[a.ld + i] = 0;
                        a.nsteps[2 * a.ld + i] = 0;
                    }
                    pass = true;
                }
            }
        }
        if (a.route) a.route[i] = pass ? 1 : 0;
    }
    // wave-aggregated append of the rejected particles to the fallback list
    const bool fail = i < a.n && !pass;
    const unsigned long long m = __ballot(fail);
    if (m) {
        const int lane = threadIdx.x & 63;
        int base = 0;
        if (lane == __ffsll((long long)m) - 1) base = atomicAdd(a.fb_count, (int)__popcll(m));
        base = __shfl(base, __ffsll((long long)m) - 1);
        if (fail) a.fb_idx[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
    }
}

__global__ void k_zero_i32(int32_t* p) { p[0] = 0; }

}  // namespace
}  // namespace adm1

using namespace adm1;

struct adm1_surrogate {
    adm1_ctx* ctx;
    int64_t n_max, batch_max;
    float* P;          // FP32 master parameters (padded layout)
    float* G;          // gradients
    float* M;          // Adam first moments
    float* V;          // Adam second moments
    uint8_t* mask;     // 1 for real parameters, 0 for padding
    uint16_t* WT;      // BF16 [out_pad][in_pad] per layer
    uint16_t* Wb;      // BF16 [in_pad][out_pad] per layer
    float* norm;       // [kMlpNorm]
    double* floor_;    // [35]
    adm1_mlp_norm host_norm;
    GateConsts gate;
    // inference
    uint16_t* X;       // [n_max][64]
    float* Y;          // [n_max][48]
    int32_t* fb_idx;   // [n_max]
    int32_t* fb_count;
    // training (batch_max rows; transposed copies [features][ldt], ldt the
    // batch rounded up to 32, for the weight-gradient GEMMs)
    float* z[4];       // pre-activations [B][256]
    uint16_t* hT[4];   // activations [256][ldt]
    uint16_t* xT;      // input [64][ldt]
    float* Yt;
    float* dY;
    uint16_t* dYb;
    uint16_t* dYT;     // [48][ldt]
    float* dH;
    float* dZ;
    uint16_t* dZb;
    uint16_t* dZT;     // [256][ldt]
    float* split;      // split-K and column-sum partials
    float* lossp;      // loss block partials
    std::vector<void*> allocs;
};

namespace {

constexpr int kSplitMax = 32;
constexpr int64_t kMlpRealParams =
    (int64_t)kMlpIn * kMlpHidden + kMlpHidden + 3 * ((int64_t)kMlpHidden * kMlpHidden + kMlpHidden) +
    (int64_t)kMlpHidden * kMlpOut + kMlpOut;
static_assert(kMlpRealParams == ADM1_MLP_PARAMS, "parameter count");

template <typename T>
bool dalloc(adm1_surrogate* s, T*& p, int64_t count)
{
    p = nullptr;
    if (count <= 0) count = 1;
    if (hipMalloc((void**)&p, (size_t)count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    try {
        s->allocs.push_back((void*)p);
    } catch (...) {
        (void)hipFree(p);
        p = nullptr;
        return false;
    }
    return true;
}

int64_t wt_offset(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)kMlpPadIn[k] * kMlpPadOut[k];
    return o;
}

// Gate constants from the model parameters (COD weights are 1 for every
// COD-bearing liquid entry; the headspace holds V_gas/V_liq per unit liquid
// volume; nitrogen contents as in the stoichiometric closure).
void gate_consts(const adm1_params& r, GateConsts& g)
{
    std::memset(g.cod_w, 0, sizeof(g.cod_w));
    std::memset(g.n_w, 0, sizeof(g.n_w));
    const int cod_rows[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 14, 15, 16, 17, 18, 19,
                            20, 21, 22, 23};
    for (int k : cod_rows) g.cod_w[k] = 1.0;
    g.cod_w[32] = r.V_gas_per_V_liq;
    g.cod_w[33] = r.V_gas_per_V_liq;
    g.n_w[10] = 1.0;             // S_IN
    g.n_w[1] = r.N_aa;           // S_aa
    g.n_w[14] = r.N_aa;          // X_pr
    g.n_w[11] = r.N_I;           // S_I
    g.n_w[23] = r.N_I;           // X_I
    g.n_w[12] = r.N_xc;          // X_xc
    for (int k = 16; k <= 22; ++k) g.n_w[k] = r.N_bac;
    for (int k = 0; k < NLIQ; ++k) {
        g.cod_in_w[k] = g.cod_w[k];
        g.n_in_w[k] = g.n_w[k];
    }
}

int check_surrogate(const adm1_surrogate* s) { return s && s->ctx ? ADM1_OK : ADM1_E_NULL; }

MlpDev mlp_dev(const adm1_surrogate* s, bool save)
{
    MlpDev m;
    for (int l = 0; l < kMlpLayers; ++l) {
        m.WT[l] = s->WT + wt_offset(l);
        m.bias[l] = s->P + mlp_b_offset(l);
    }
    for (int l = 0; l < 4; ++l) {
        m.z[l] = save ? s->z[l] : nullptr;
        m.hT[l] = save ? s->hT[l] : nullptr;
    }
    m.xT = save ? s->xT : nullptr;
    m.ldt = 0;
    return m;
}

hipError_t repack(adm1_surrogate* s, hipStream_t st)
{
    for (int l = 0; l < kMlpLayers; ++l) {
        const hipError_t e = pack(s->P + mlp_w_offset(l), kMlpPadIn[l], kMlpPadOut[l],
                                  s->WT + wt_offset(l), s->Wb + wt_offset(l), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int adm1_surrogate_create(adm1_ctx* ctx, int64_t n_max, int64_t batch_max, adm1_surrogate** out)
{
    if (!ctx || !out) return ADM1_E_NULL;
    if (n_max < 0 || batch_max < 0 || n_max > ctx->n_max || n_max > INT32_MAX)
        return ADM1_E_SIZE;
    adm1_surrogate* s = new (std::nothrow) adm1_surrogate;
    if (!s) return ADM1_E_NOMEM;
    s->ctx = ctx;
    s->n_max = n_max;
    s->batch_max = batch_max;
    std::memset(&s->host_norm, 0, sizeof(s->host_norm));
    std::memset(&s->gate, 0, sizeof(s->gate));
    gate_consts(ctx->raw, s->gate);
    const int64_t np = kMlpPadParams;
    const int64_t nw = wt_offset(kMlpLayers);
    const int64_t B = batch_max;
    const int64_t split = (int64_t)kSplitMax * kMlpHidden * kMlpHidden;
    bool ok = dalloc(s, s->P, np) && dalloc(s, s->G, np) && dalloc(s, s->M, np) &&
              dalloc(s, s->V, np) && dalloc(s, s->mask, np) && dalloc(s, s->WT, nw) &&
              dalloc(s, s->Wb, nw) && dalloc(s, s->norm, kMlpNorm) &&
              dalloc(s, s->floor_, NX) && dalloc(s, s->X, n_max * kMlpInPad) &&
              dalloc(s, s->Y, n_max * kMlpOutPad) && dalloc(s, s->fb_idx, n_max) &&
              dalloc(s, s->fb_count, 64);
    const int64_t ldt = (B + 31) / 32 * 32;
    for (int l = 0; l < 4 && ok; ++l)
        ok = dalloc(s, s->z[l], B * kMlpHidden) && dalloc(s, s->hT[l], ldt * kMlpHidden);
    ok = ok && dalloc(s, s->xT, ldt * kMlpInPad) && dalloc(s, s->Yt, B * kMlpOutPad) &&
         dalloc(s, s->dY, B * kMlpOutPad) && dalloc(s, s->dYb, B * kMlpOutPad) &&
         dalloc(s, s->dYT, ldt * kMlpOutPad) && dalloc(s, s->dH, B * kMlpHidden) &&
         dalloc(s, s->dZ, B * kMlpHidden) && dalloc(s, s->dZb, B * kMlpHidden) &&
         dalloc(s, s->dZT, ldt * kMlpHidden) && dalloc(s, s->split, split) &&
         dalloc(s, s->lossp, (B * kMlpOutPad + 255) / 256 + 1);
    if (ok) try {
        // zero parameters and moments; mask of the real entries
        std::vector<uint8_t> mask((size_t)np, 0);
        for (int l = 0; l < kMlpLayers; ++l) {
            for (int r = 0; r < kMlpDimIn[l]; ++r)
                for (int c = 0; c < kMlpDimOut[l]; ++c)
                    mask[(size_t)(mlp_w_offset(l) + (int64_t)r * kMlpPadOut[l] + c)] = 1;
            for (int c = 0; c < kMlpDimOut[l]; ++c) mask[(size_t)(mlp_b_offset(l) + c)] = 1;
        }
        ok = hipMemset(s->P, 0, np * sizeof(float)) == hipSuccess &&
             hipMemset(s->G, 0, np * sizeof(float)) == hipSuccess &&
             hipMemset(s->M, 0, np * sizeof(float)) == hipSuccess &&
             hipMemset(s->V, 0, np * sizeof(float)) == hipSuccess &&
             hipMemset(s->WT, 0, nw * sizeof(uint16_t)) == hipSuccess &&
             hipMemset(s->Wb, 0, nw * sizeof(uint16_t)) == hipSuccess &&
             hipMemset(s->norm, 0, kMlpNorm * sizeof(float)) == hipSuccess &&
             hipMemset(s->floor_, 0, NX * sizeof(double)) == hipSuccess &&
             hipMemcpy(s->mask, mask.data(), (size_t)np, hipMemcpyHostToDevice) == hipSuccess;
    } catch (...) {
        ok = false;
    }
    if (!ok) {
        (void)hipGetLastError();
        adm1_surrogate_destroy(s);
        return ADM1_E_NOMEM;
    }
    *out = s;
    return ADM1_OK;
}

void adm1_surrogate_destroy(adm1_surrogate* s)
{
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
}

int adm1_surrogate_set_weights(adm1_surrogate* s, const float* params, const adm1_mlp_norm* norm)
try {
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!params || !norm) return ADM1_E_NULL;
    for (int k = 0; k < kMlpIn; ++k)
        if (!(norm->in_sd[k] > 0.0f) || !std::isfinite(norm->in_mean[k])) return ADM1_E_PARAMS;
    for (int k = 0; k < kMlpOut; ++k)
        if (!(norm->out_sd[k] > 0.0f) || !std::isfinite(norm->out_mean[k]) ||
            !(norm->floor[k] > 0.0))
            return ADM1_E_PARAMS;
    std::vector<float> pad((size_t)kMlpPadParams, 0.0f);
    const float* src = params;
    for (int l = 0; l < kMlpLayers; ++l) {
        for (int r = 0; r < kMlpDimIn[l]; ++r)
            for (int c = 0; c < kMlpDimOut[l]; ++c)
                pad[(size_t)(mlp_w_offset(l) + (int64_t)r * kMlpPadOut[l] + c)] = *src++;
        for (int c = 0; c < kMlpDimOut[l]; ++c) pad[(size_t)(mlp_b_offset(l) + c)] = *src++;
    }
    for (float v : pad)
        if (!std::isfinite(v)) return ADM1_E_PARAMS;
    float nv[kMlpNorm];
    std::memcpy(nv, norm->in_mean, sizeof(norm->in_mean));
    std::memcpy(nv + kMlpIn, norm->in_sd, sizeof(norm->in_sd));
    std::memcpy(nv + 2 * kMlpIn, norm->out_mean, sizeof(norm->out_mean));
    std::memcpy(nv + 2 * kMlpIn + kMlpOut, norm->out_sd, sizeof(norm->out_sd));
    const size_t nb = (size_t)kMlpPadParams * sizeof(float);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(s->P, pad.data(), nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->M, 0, nb) != hipSuccess || hipMemset(s->V, 0, nb) != hipSuccess ||
        hipMemset(s->G, 0, nb) != hipSuccess ||
        hipMemcpy(s->norm, nv, sizeof(nv), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->floor_, norm->floor, sizeof(norm->floor), hipMemcpyHostToDevice) !=
            hipSuccess)
        return hip_rc(hipGetLastError());
    s->host_norm = *norm;
    for (int k = 0; k < kMlpOut; ++k) {
        s->gate.out_mean[k] = norm->out_mean[k];
        s->gate.out_sd[k] = norm->out_sd[k];
        s->gate.floor_[k] = norm->floor[k];
    }
    rc = hip_rc(repack(s, nullptr));
    if (rc) return rc;
    return hip_rc(hipDeviceSynchronize());
} catch (...) {
    return ADM1_E_NOMEM;
}

int adm1_surrogate_get_weights(adm1_surrogate* s, float* params, adm1_mlp_norm* norm)
try {
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (params) {
        std::vector<float> pad((size_t)kMlpPadParams);
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(pad.data(), s->P, pad.size() * sizeof(float), hipMemcpyDeviceToHost) !=
                hipSuccess)
            return hip_rc(hipGetLastError());
        float* dst = params;
        for (int l = 0; l < kMlpLayers; ++l) {
            for (int r = 0; r < kMlpDimIn[l]; ++r)
                for (int c = 0; c < kMlpDimOut[l]; ++c)
                    *dst++ = pad[(size_t)(mlp_w_offset(l) + (int64_t)r * kMlpPadOut[l] + c)];
            for (int c = 0; c < kMlpDimOut[l]; ++c) *dst++ = pad[(size_t)(mlp_b_offset(l) + c)];
        }
    }
    if (norm) *norm = s->host_norm;
    return ADM1_OK;
} catch (...) {
    return ADM1_E_NOMEM;
}

int adm1_surrogate_get_grads(adm1_surrogate* s, float* grads)
try {
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!grads) return ADM1_E_NULL;
    std::vector<float> pad((size_t)kMlpPadParams);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(pad.data(), s->G, pad.size() * sizeof(float), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return hip_rc(hipGetLastError());
    float* dst = grads;
    for (int l = 0; l < kMlpLayers; ++l) {
        for (int r = 0; r < kMlpDimIn[l]; ++r)
            for (int c = 0; c < kMlpDimOut[l]; ++c)
                *dst++ = pad[(size_t)(mlp_w_offset(l) + (int64_t)r * kMlpPadOut[l] + c)];
        for (int c = 0; c < kMlpDimOut[l]; ++c) *dst++ = pad[(size_t)(mlp_b_offset(l) + c)];
    }
    return ADM1_OK;
} catch (...) {
    return ADM1_E_NOMEM;
}

int adm1_surrogate_featurize(adm1_surrogate* s, const double* state, int64_t ld,
                             const double* temp_K, const double* D, double dt_days, int64_t n,
                             uint16_t* X, void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!state || !temp_K || !D || !X) return ADM1_E_NULL;
    if ((rc = check_layout(s->ctx, ld, n))) return rc;
    if (((uintptr_t)X & 15) != 0) return ADM1_E_SIZE;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    if (!is_device(state) || !is_device(temp_K) || !is_device(D) || !is_device(X))
        return ADM1_E_NOT_DEVICE;
    return hip_rc(featurize(state, ld, temp_K, D, dt_days, n, s->norm, s->floor_, X,
                            (hipStream_t)stream));
}

int adm1_surrogate_targets(adm1_surrogate* s, const double* x0, const double* x1, int64_t ld,
                           int64_t n, float* target, void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!x0 || !x1 || !target) return ADM1_E_NULL;
    if ((rc = check_layout(s->ctx, ld, n))) return rc;
    if (!is_device(x0) || !is_device(x1) || !is_device(target)) return ADM1_E_NOT_DEVICE;
    return hip_rc(targets(x0, x1, ld, n, s->norm, s->floor_, target, (hipStream_t)stream));
}

int adm1_surrogate_forward(adm1_surrogate* s, const uint16_t* X, int64_t n, float* Y,
                           void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!X || !Y) return ADM1_E_NULL;
    if (n < 0 || ((uintptr_t)X & 15) != 0) return ADM1_E_SIZE;
    if (!is_device(X) || !is_device(Y)) return ADM1_E_NOT_DEVICE;
    return hip_rc(mlp_forward(mlp_dev(s, false), X, n, Y, false, (hipStream_t)stream));
}

int adm1_surrogate_gate(adm1_surrogate* s, double* state, int64_t ld, const double* temp_K,
                        const adm1_feed* feed, double dt_days, int64_t n, const float* Y,
                        const adm1_gate* gate, adm1_aux* aux, uint8_t* status, int32_t* nsteps,
                        uint8_t* route, int32_t* fb_idx, int32_t* fb_count, void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!state || !temp_K || !Y || !gate || !status || !fb_idx || !fb_count) return ADM1_E_NULL;
    if ((rc = check_layout(s->ctx, ld, n))) return rc;
    if (n > INT32_MAX) return ADM1_E_SIZE;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    if ((rc = check_feed_no_phase(feed))) return rc;  // the surrogate models no phases
    if (!(gate->max_dlog >= 0.0) || !(gate->tol_ion >= 0.0) || !(gate->tol_closure >= 0.0))
        return ADM1_E_OPTS;
    if (!is_device(state) || !is_device(temp_K) || !is_device(Y) || !is_device(status) ||
        !is_device(fb_idx) || !is_device(fb_count))
        return ADM1_E_NOT_DEVICE;
    if ((nsteps && !is_device(nsteps)) || (route && !is_device(route)))
        return ADM1_E_NOT_DEVICE;
    if (aux && aux->H && !is_device(aux->H)) return ADM1_E_NOT_DEVICE;
    GateArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = s->ctx->dp;
    a.g = s->gate;
    a.g.max_dlog = gate->max_dlog;
    a.g.tol_ion = gate->tol_ion;
    a.g.tol_closure = gate->tol_closure;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.dt = dt_days; a.Y = Y;
    a.H = aux ? aux->H : nullptr;
    a.status = status; a.nsteps = nsteps; a.route = route; a.fb_idx = fb_idx;
    a.fb_count = fb_count;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, fb_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_rc(e);
    if (n == 0) return ADM1_OK;
    hipLaunchKernelGGL(k_gate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    return hip_rc(hipGetLastError());
}

int adm1_surrogate_step(adm1_surrogate* s, double* state, int64_t ld, const double* temp_K,
                        const adm1_feed* feed, double dt_days, int64_t n, const adm1_gate* gate,
                        adm1_aux* aux, uint8_t* status, int32_t* nsteps, uint8_t* route,
                        int32_t* fb_count, void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if ((rc = check_feed_no_phase(feed))) return rc;  // the surrogate models no phases
    if (n > s->n_max) return ADM1_E_SIZE;
    if (fb_count && !is_device(fb_count)) return ADM1_E_NOT_DEVICE;
    if (aux && aux->h_last && !is_device(aux->h_last)) return ADM1_E_NOT_DEVICE;
    int32_t* cnt = fb_count ? fb_count : s->fb_count;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = adm1_surrogate_featurize(s, state, ld, temp_K, feed->D, dt_days, n, s->X, stream)))
        return rc;
    if (n > 0) {
        rc = hip_rc(mlp_forward(mlp_dev(s, false), s->X, n, s->Y, false, st));
        if (rc) return rc;
    }
    if ((rc = adm1_surrogate_gate(s, state, ld, temp_K, feed, dt_days, n, s->Y, gate, aux,
                                  status, nsteps, route, s->fb_idx, cnt, stream)))
        return rc;
    if (n == 0) return hip_rc(adm1::launch_count_status(status, 0, s->ctx->d_fail, st));
    adm1_ctx* ctx = s->ctx;
    adm1::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = ctx->dp;
    a.state = state; a.ld = ld; a.n = n; a.T = temp_K; a.D = feed->D; a.fidx = feed->idx;
    a.S_in = feed->S_in; a.n_feed = feed->n_feed; a.dt = dt_days;
    a.H = aux ? aux->H : nullptr;
    a.hlast = aux ? aux->h_last : nullptr;
    a.status = status; a.nsteps = nsteps; a.queue = ctx->d_queue;
    a.index = s->fb_idx; a.index_count = cnt;
    a.pdev = ctx->d_params;
    a.service_batch = ctx->tuned_service_batch;
    // the fallback list in expected-cost order, as the full step orders its
    // queue (rejected particles are the stiff ones: the tail matters most)
    if (ctx->order_mode == ADM1_ORDER_COST && a.hlast) {
        rc = hip_rc(adm1::launch_cost_order(a.hlast, s->fb_idx, cnt, n, dt_days,
                                            ctx->d_order_work, ctx->d_order, st));
        if (rc) return rc;
        a.index = ctx->d_order;
        a.index_count = ctx->d_order_work + 2 * adm1::kOrderBuckets;
    }
    rc = hip_rc(adm1::launch_step_sparse2(a, ctx->opts.rate_precision, ctx->tuned_blocks_per_cu,
                                          st));
    if (rc) return rc;
    return hip_rc(adm1::launch_count_status(status, n, ctx->d_fail, st));
}

int adm1_surrogate_graph_capture_step(adm1_surrogate* s, double* state, int64_t ld,
                                      const double* temp_K, const adm1_feed* feed,
                                      double dt_days, int64_t n, const adm1_gate* gate,
                                      adm1_aux* aux, uint8_t* status, int32_t* nsteps,
                                      uint8_t* route, int32_t* fb_count, const double* V_liq,
                                      double* q_gas, double* q_ch4, double* totals,
                                      void* stream, adm1_graph** out)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!out || !stream || !feed || !gate) return ADM1_E_NULL;
    if ((rc = check_feed_no_phase(feed))) return rc;  // the surrogate models no phases
    if (n < 0 || n > s->n_max) return ADM1_E_SIZE;
    if (!(gate->max_dlog >= 0.0) || !(gate->tol_ion >= 0.0) || !(gate->tol_closure >= 0.0))
        return ADM1_E_OPTS;
    // validate the step's arguments before capturing (n = 0 enqueues nothing)
    if ((rc = adm1_step_particles(s->ctx, state, ld, temp_K, feed, dt_days, 0, aux, status,
                                  nsteps, stream)))
        return rc;
    if (!totals) return ADM1_E_NULL;
    adm1_graph* g = new (std::nothrow) adm1_graph;
    if (!g) return ADM1_E_NOMEM;
    g->graph = nullptr;
    g->exec = nullptr;
    hipStream_t st = (hipStream_t)stream;
    const hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        delete g;
        return (int)e;
    }
    rc = adm1_surrogate_step(s, state, ld, temp_K, feed, dt_days, n, gate, aux, status, nsteps,
                             route, fb_count, stream);
    if (rc == ADM1_OK)
        rc = adm1_gas_flux(s->ctx, state, ld, temp_K, V_liq, n, q_gas, q_ch4, totals, stream);
    return finish_capture(st, rc, g, out);
}

int adm1_surrogate_train_step(adm1_surrogate* s, const uint16_t* X, const float* target,
                              int64_t B, float lr, int32_t step, float* loss, void* stream)
{
    int rc = check_surrogate(s);
    if (rc) return rc;
    if (!X || !target || !loss) return ADM1_E_NULL;
    if (B < 1 || B > s->batch_max || B > INT32_MAX / kMlpHidden) return ADM1_E_SIZE;
    if (step < 1 || !(lr >= 0.0f) || !std::isfinite(lr)) return ADM1_E_OPTS;
    if (!is_device(X) || !is_device(target) || !is_device(loss)) return ADM1_E_NOT_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    const int64_t ldt = (B + 31) / 32 * 32;
    MlpDev md = mlp_dev(s, true);
    md.ldt = ldt;
    hipError_t e = mlp_forward(md, X, B, s->Yt, true, st);
    if (e == hipSuccess)
        e = mlp_loss(s->Yt, target, B, ldt, s->dY, s->dYb, s->dYT, s->lossp, loss, st);
    const int Bi = (int)B;
    const int splitk = (int)std::min<int64_t>(kSplitMax, std::max<int64_t>(1, ldt / 256));
    // backward, last layer first; dZ of layer l is (dY, dYb, dYT) for l = 4
    for (int l = kMlpLayers - 1; l >= 0 && e == hipSuccess; --l) {
        const int I = kMlpPadIn[l], O = kMlpPadOut[l];
        const uint16_t* AinT = l == 0 ? s->xT : s->hT[l - 1];
        const bool top = l == kMlpLayers - 1;
        const float* dZf = top ? s->dY : s->dZ;
        const uint16_t* dZh = top ? s->dYb : s->dZb;
        const uint16_t* dZT = top ? s->dYT : s->dZT;
        // dW = A_in^T dZ  ([I][O], contraction over the batch)
        e = gemm_tn(AinT, ldt, dZT, ldt, s->G + mlp_w_offset(l), O, I, O, (int)ldt, splitk,
                    s->split, st);
        if (e == hipSuccess) e = colsum(dZf, B, O, O, s->G + mlp_b_offset(l), s->split, st);
        if (l == 0 || e != hipSuccess) continue;
        // dH = dZ W^T ([B][I]), then through the GELU of layer l - 1
        e = gemm_tn(dZh, O, s->Wb + wt_offset(l), O, s->dH, I, Bi, I, O, 1, nullptr, st);
        if (e == hipSuccess)
            e = gelu_bwd(s->dH, s->z[l - 1], B, ldt, s->dZ, s->dZb, s->dZT, st);
    }
    if (e == hipSuccess)
        e = adam(s->P, s->G, s->M, s->V, s->mask, kMlpPadParams, lr, 0.9f, 0.999f, 1e-8f, step,
                 st);
    if (e == hipSuccess) e = repack(s, st);
    return hip_rc(e);
}

}  // extern "C"
