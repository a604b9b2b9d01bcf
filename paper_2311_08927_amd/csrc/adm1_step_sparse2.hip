// Two-lanes-per-particle ADM1 step for gfx950: register-resident sparse LU.
//
// Each particle is integrated over one coupling interval (sec. 2.3) by the
// adaptive Rodas4 step of adm1_rodas4.h on the 28 differential entries, the
// eq. 7 and eq. 8 unknowns being eliminated through the bordered Newton
// matrix.  A particle's live state (a 242-entry LU, five stage vectors, the
// right-hand-side temporaries) exceeds one lane's registers, so a lane PAIR
// owns one particle:
//   - the LU rows are split over the pair (gen_jac.py pairs rows of similar
//     pattern) and stay in registers; pivot rows and solution components
//     cross the pair with DPP quad_perm broadcasts, so both lanes run one
//     instruction stream;
//   - each lane keeps its rows' components of the stage vectors and the
//     pair's whole stage argument in LDS (40 KB per wave, so four waves,
//     one per SIMD, fit a compute unit) and its rows of the state in
//     registers; the LU and the rates fill the rest of the registers (what
//     still spills is the only per-step memory traffic).  Four stage
//     vectors are stored: the fifth stage folds u_1..u_5 into the argument
//     and correction sums the sixth stage needs, which replace u_1, u_2;
//   - inflow terms D S_in are read from the (small, cached) feed table;
//   - both lanes evaluate the right-hand side redundantly (it needs the whole
//     state) and each keeps only its rows of it;
//   - the algebraic solves of each stage start from the linear prediction
//     z0 + sum_j a_ij w_j, w_j the constraint components of the bordered
//     stage solutions.
// The kernel is persistent: pairs that finish their particle fetch the next
// one from a global counter (wave-aggregated atomics), so particles with
// many steps (feed-zone pulses, cold starts) do not idle the others.
#include <hip/hip_runtime.h>

#include "adm1_kernels.h"
#include "adm1_model.h"
#include "adm1_rodas4.h"
#include <adm1_jac_sparse2.inc>

namespace adm1 {

namespace {

constexpr int NP = ADM1_SP2_NPAIR;  // 15 row pairs (the last one: eq. 7 / eq. 8 rows)
constexpr int NDP = NP - 1;         // 14 pairs of differential rows
constexpr int kVar0[NP] = ADM1_SP2_PAIR_VAR0;
constexpr int kVar1[NP] = ADM1_SP2_PAIR_VAR1;
constexpr int kVarPair[NP * 2] = ADM1_SP2_VAR_PAIR;
constexpr int kVarSide[NP * 2] = ADM1_SP2_VAR_SIDE;
constexpr int kWavesPerCU = 4;  // one wave per SIMD: 4 x 40 KB of LDS per CU
constexpr int kStored = 4;      // stage vectors kept in LDS (see the header)
constexpr int kServiceBatch = 4;  // pairs served per service pass (default)
static_assert(kR4Stages == 6, "the stage-5 accumulation assumes six stages");

static_assert(kVar0[NP - 1] == 28 && kVar1[NP - 1] == 29,
              "the constraint rows must form the last pair");

// Parameter block in the constant address space; laundering the pointer
// keeps the compiler from hoisting ~200 uniform parameters into spilled
// scalar registers: they are re-read (scalar cache) where they are used.
typedef __attribute__((address_space(4))) const DevParams* cparams_t;
__device__ __forceinline__ const DevParams& params_at(cparams_t pp)
{
    asm volatile("" : "+s"(pp));
    return *(const DevParams*)pp;
}

// quad_perm DPP: each lane of a pair takes lane (lane & ~1) + SRC.
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double bc0(double v) { return dpp<0xA0>(v); }  // [0,0,2,2]
__device__ __forceinline__ double bc1(double v) { return dpp<0xF5>(v); }  // [1,1,3,3]
__device__ __forceinline__ double swp(double v) { return dpp<0xB1>(v); }  // [1,0,3,2]

// Full 28-vector on both lanes from the pair's own components.
__device__ __forceinline__ void gather(const double* own, double* full, bool odd)
{
#pragma unroll
    for (int m = 0; m < NDP; ++m) {
        const double other = swp(own[m]);
        full[kVar0[m]] = odd ? other : own[m];
        full[kVar1[m]] = odd ? own[m] : other;
    }
}

// Shared memory of one wave (one block of 64 lanes = 32 particle pairs).
struct Lds {
    double u[kStored][NDP][64];         // own components of the stage vectors
    double tc[10][32];                  // temperature constants (9) and D per pair
    double w[kR4Stages - 1][2][32];     // constraint components of the stage solutions
    double arg[NY][32];                 // current stage argument (whole vector) per pair
};

// Whole stage argument of a pair, read from LDS where the rates use it.
struct LdsVec {
    const Lds* L;
    int pr;
    __device__ __forceinline__ double operator[](int k) const { return L->arg[k][pr]; }
};

__device__ __forceinline__ TConst load_tc(const Lds& L, int pr)
{
    TConst c;
    c.RT = L.tc[0][pr]; c.K_w = L.tc[1][pr]; c.K_a_co2 = L.tc[2][pr];
    c.K_a_IN = L.tc[3][pr]; c.K_H_h2 = L.tc[4][pr]; c.K_H_ch4 = L.tc[5][pr];
    c.K_H_co2 = L.tc[6][pr]; c.p_h2o = L.tc[7][pr]; c.arr = L.tc[8][pr];
    return c;
}

// The starting step's root (cold starts only) kept out of line, so that the
// constants of exp/log are not hoisted into the persistent loop.  It is
// called only where every lane of the wave is active: a call made under a
// partial exec mask may overwrite the values the inactive lanes hold in
// caller-saved registers (measured: warm-start guesses of waiting pairs
// changed, making a particle's rounding depend on its neighbours).
__device__ __attribute__((noinline)) double fifth_root(double x)
{
    return exp(0.2 * log(x));
}

// Inflow terms D S_in seen by one lane's right-hand side: only the lane's
// own rows are assembled (the partner's are discarded), so only those and the
// S_h2 inflow of eq. 8 are loaded; the accessor takes a state row.
struct PairInflow {
    double own[NDP];
    double sh2;
    bool odd;
    __device__ __forceinline__ double operator()(int row) const
    {
        if (row == ROW_SH2) return sh2;
        const int k = row < ROW_SH2 ? row : row - 1;   // integration index
        return ((kVarSide[k] != 0) == odd) ? own[kVarPair[k]] : 0.0;
    }
};

__device__ __forceinline__ PairInflow pair_inflow(const double* sin, double D, bool odd)
{
    PairInflow f;
    f.odd = odd;
#pragma unroll
    for (int m = 0; m < NDP; ++m) {
        const int k0 = kVar0[m], k1 = kVar1[m];
        const int r0 = k0 <= San ? state_row(k0) : -1;
        const int r1 = k1 <= San ? state_row(k1) : -1;
        const int r = odd ? r1 : r0;
        f.own[m] = r >= 0 ? D * sin[r >= 0 ? r : 0] : 0.0;
    }
    f.sh2 = D * sin[ROW_SH2];
    return f;
}

// Per-pair integration state kept in registers across loop iterations.
struct PairState {
    double t, h, H, Sh2, hlast;
    int64_t pid;
    int n, acc, rej, it, fi;
    bool reject_prev;
    double y[NDP];  // own components of the particle's state
};

enum Job { kNone = 0, kFinish = 1, kStart = 2, kHinit = 3, kRoot = 4 };

__device__ __forceinline__ void write_status(const StepArgs& a, const PairState& s, int st,
                                             bool odd)
{
    if (!odd) {
        const int64_t i = s.pid;
        a.status[i] = (uint8_t)st;
        if (a.nsteps) {
            a.nsteps[i] = s.acc;
            a.nsteps[a.ld + i] = s.rej;
            a.nsteps[2 * a.ld + i] = s.it;
        }
    }
}

// Service loop: particles that finished their interval are written back,
// free pairs fetch new particles (wave-aggregated atomics on the queue) and
// start them (load, checks, algebraic solve at y0, starting step).  One
// right-hand-side site serves every job.  On exit every pair is active or
// the queue is exhausted for it.
template <typename R>
__device__ static void service(const StepArgs& a, cparams_t pp, Lds& L, PairState& s,
                               int& job, int fin_status, bool& active, bool& exhausted,
                               bool odd_in, int lane_in, int64_t total)
{
    int lane = lane_in;
    asm volatile("" : "+v"(lane));
    const bool odd = lane & 1;
    const int pr = lane >> 1;
    double yin[NY], f[NY], f0[NY];
    double h0 = 0.0, d1 = 0.0, dm = 0.0;
    for (;;) {
        const bool need = !active && !exhausted && job == kNone;
        const unsigned long long needm = __ballot(need && !odd);
        if (needm) {
            int base = 0;
            if (lane == 0) base = atomicAdd(a.queue, (int)__popcll(needm));
            base = __shfl(base, 0);
            if (need) {
                const int rank = __popcll(needm & ((1ull << (lane & ~1)) - 1ull));
                const int64_t q = (int64_t)base + rank;
                if (q < total) {
                    s.pid = a.index ? (int64_t)a.index[q] : q;
                    job = kStart;
                } else {
                    exhausted = true;
                }
            }
        }
        if (!__any(job != kNone)) break;
        // the out-of-line root of the starting-step estimate, here with every
        // lane active (the condition is wave-uniform, so the exec mask stays
        // full)
        double root = 1.0;
        if (__any(job == kRoot)) root = fifth_root(job == kRoot ? 0.01 / dm : 1.0);
        if (job == kRoot) {
            const double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : root;
            s.h = fmin(fmin(100.0 * h0, h1), a.dt);
            active = true;
            job = kNone;
        }
        if (job == kNone) continue;
        const DevParams& p = params_at(pp);
        const int64_t i = s.pid;
        bool run = true;
        TConst c;
        double D;
        if (job == kFinish) {
            if (fin_status != 0) {
                write_status(a, s, fin_status, odd);
                job = kNone;
                run = false;
            } else {
                double own[NDP];
#pragma unroll
                for (int m = 0; m < NDP; ++m) own[m] = s.y[m];
                gather(own, yin, odd);
            }
            c = load_tc(L, pr);
            D = L.tc[9][pr];
        } else if (job == kStart) {
#pragma unroll
            for (int k = 0; k < NY; ++k) yin[k] = a.state[state_row(k) * a.ld + i];
            const double T = a.T[i];
            D = a.D[i];
            const int fi = a.fidx[i];
            s.H = a.H ? a.H[i] : -1.0;
            s.hlast = a.hlast ? a.hlast[i] : -1.0;
            s.Sh2 = a.state[ROW_SH2 * a.ld + i];
            s.n = s.acc = s.rej = s.it = 0;
            s.fi = fi;
            s.t = 0.0;
            s.reject_prev = false;
            bool fin = isfinite(T) && T > 0.0 && isfinite(D) && fi >= 0 && fi < a.n_feed;
#pragma unroll
            for (int k = 0; k < NY; ++k) fin = fin & isfinite(yin[k]);
            const double* sin = a.S_in + (int64_t)(fin ? fi : 0) * NLIQ;
            if (fin) {
#pragma unroll
                for (int k = 0; k < NLIQ; ++k) fin = fin & isfinite(sin[k]);
            }
            if (!fin) {
                write_status(a, s, 4, odd);
                job = kNone;
                run = false;
            } else {
                c = tconst(p, T);
                c.arr *= phase_factor(a.phase, a.phase_kin, i);
                if (!odd) {
                    L.tc[0][pr] = c.RT; L.tc[1][pr] = c.K_w; L.tc[2][pr] = c.K_a_co2;
                    L.tc[3][pr] = c.K_a_IN; L.tc[4][pr] = c.K_H_h2; L.tc[5][pr] = c.K_H_ch4;
                    L.tc[6][pr] = c.K_H_co2; L.tc[7][pr] = c.p_h2o; L.tc[8][pr] = c.arr;
                    L.tc[9][pr] = D;
                }
                if (s.hlast > 0.0 && s.H > 0.0) {
                    // warm start: the input's algebraic entries and S_H+ are
                    // the previous interval's solution at this state, and the
                    // first stage solves eqs. 7-8 from them; no separate
                    // evaluation at y0 is needed (a failure there is reported
                    // as at the interval start)
#pragma unroll
                    for (int m = 0; m < NDP; ++m)
                        s.y[m] = odd ? yin[kVar1[m]] : yin[kVar0[m]];
                    s.h = fmin(a.dt, s.hlast);
                    active = true;
                    job = kNone;
                    run = false;
                }
            }
        } else {  // kHinit: second evaluation of the starting-step estimate
#pragma unroll
            for (int k = 0; k < NY; ++k) yin[k] = f0[k] * h0 + yin[k];
            c = load_tc(L, pr);
            D = L.tc[9][pr];
        }
        if (!run) continue;
        double Ht = s.H, St = s.Sh2;
        // the end of the interval needs only the algebraic entries
        const int rc = rhs_in<R>(p, c, yin, D, FeedInflow{D, a.S_in + (int64_t)s.fi * NLIQ},
                                 Ht, St,
                                 [&f](int k, double v) { f[k] = v; }, s.it, job == kFinish);
        if (job == kFinish) {
            int st = 0;
            if (rc) {
                st = 1;
            } else {
                const double H = Ht;
#pragma unroll
                for (int m = 0; m < NDP; ++m) {
                    const int k = odd ? kVar1[m] : kVar0[m];
                    a.state[state_row(k) * a.ld + i] = s.y[m];
                }
                if (!odd) {
                    a.state[ROW_SH2 * a.ld + i] = St;
                    a.state[26 * a.ld + i] = p.K_a_va * yin[Sva] / (p.K_a_va + H);
                    a.state[27 * a.ld + i] = p.K_a_bu * yin[Sbu] / (p.K_a_bu + H);
                    a.state[28 * a.ld + i] = p.K_a_pro * yin[Spro] / (p.K_a_pro + H);
                    if (a.H) a.H[i] = H;
                    if (a.hlast) a.hlast[i] = s.hlast;
                } else {
                    a.state[29 * a.ld + i] = p.K_a_ac * yin[Sac] / (p.K_a_ac + H);
                    a.state[30 * a.ld + i] = c.K_a_co2 * yin[SIC] / (c.K_a_co2 + H);
                    a.state[31 * a.ld + i] = c.K_a_IN * yin[SIN] / (c.K_a_IN + H);
                }
                bool neg = false;
#pragma unroll
                for (int k = 0; k < NY; ++k) neg = neg | (yin[k] < 0.0);
                if (neg) st |= 0x80;
            }
            write_status(a, s, st, odd);
            job = kNone;
        } else if (job == kStart) {
            if (rc) {
                write_status(a, s, 1, odd);
                job = kNone;
            } else {
                s.H = Ht;
                s.Sh2 = St;
#pragma unroll
                for (int m = 0; m < NDP; ++m)
                    s.y[m] = odd ? yin[kVar1[m]] : yin[kVar0[m]];
                if (s.hlast > 0.0) {
                    s.h = fmin(a.dt, s.hlast);
                    active = true;
                    job = kNone;
                } else {
                    // starting step (Hairer, Norsett & Wanner, Solving ODEs I,
                    // sec. II.4), order 4: first evaluation
                    double d0 = 0.0;
                    d1 = 0.0;
#pragma unroll
                    for (int k = 0; k < NY; ++k) {
                        const double sc = p.atol[k] + p.rtol * fabs(yin[k]);
                        d0 += (yin[k] / sc) * (yin[k] / sc);
                        d1 += (f[k] / sc) * (f[k] / sc);
                        f0[k] = f[k];
                    }
                    d0 = sqrt(d0 / NY);
                    d1 = sqrt(d1 / NY);
                    h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                    if (h0 > a.dt) h0 = a.dt;
                    job = kHinit;
                }
            }
        } else {  // kHinit
            if (!rc) {
                double d2 = 0.0;
#pragma unroll
                for (int k = 0; k < NY; ++k) {
                    const double y0k = yin[k] - h0 * f0[k];
                    const double sc = p.atol[k] + p.rtol * fabs(y0k);
                    const double v = f[k] - f0[k];
                    d2 += (v / sc) * (v / sc);
                }
                d2 = sqrt(d2 / NY) / h0;
                dm = fmax(d1, d2);
                job = kRoot;  // the fifth root, at the next pass's uniform call
            } else {
                s.h = h0;
                active = true;
                job = kNone;
            }
        }
    }
}

#define b0 bv[0]
#define b1 bv[1]
#define b2 bv[2]
#define b3 bv[3]
#define b4 bv[4]
#define b5 bv[5]
#define b6 bv[6]
#define b7 bv[7]
#define b8 bv[8]
#define b9 bv[9]
#define b10 bv[10]
#define b11 bv[11]
#define b12 bv[12]
#define b13 bv[13]
#define b14 bv[14]

// One Rodas4 attempt of the pair's particle.  Returns 0 to continue, or the
// final status + 1 once the interval is done or failed.  The stage loop is
// not unrolled: one right-hand-side, factorisation and solve site.
template <typename R>
__device__ static int attempt(const StepArgs& a, cparams_t pp, Lds& L, PairState& s,
                              bool odd_in, int lane_in)
{
    // lane-dependent values (row selections, LDS offsets) are recomputed
    // here rather than kept live across the persistent loop
    int lane = lane_in;
    asm volatile("" : "+v"(lane));
    const bool odd = lane & 1;
    const int pr = lane >> 1;
    {
        const DevParams& p = params_at(pp);
        if (s.n >= p.max_steps) return 3 + 1;
    }
    if (s.h < 1e-14 * a.dt) return 2 + 1;
    double hs = s.h;
    bool clip = false;
    if (s.t + 1.01 * hs >= a.dt) {
        hs = a.dt - s.t;
        clip = true;
    }
    const double ih = frcp(hs);
    double bv[NP];
    ADM1_SP2_DECL;
    bool ok = true;
    double H0 = s.H, S0 = s.Sh2;
    // Stage vectors (this lane's row-pair components) in L.u: u_j in slot j
    // for j < 4; after the fifth stage, slot 0 holds sum_j a_6j u_j and
    // slot 1 sum_j c_6j u_j (j < 5).
#pragma unroll 1
    for (int st = 0; st < kR4Stages; ++st) {
        const LdsVec arg{&L, pr};
        {
            double own[NDP];
#pragma unroll
            for (int m = 0; m < NDP; ++m) own[m] = s.y[m];
            if (st < kR4Stages - 1) {
                for (int j = 0; j < st; ++j) {
                    const double aj = kR4A[st][j];
#pragma unroll
                    for (int m = 0; m < NDP; ++m) own[m] += aj * L.u[j][m][lane];
                }
            } else {
#pragma unroll
                for (int m = 0; m < NDP; ++m) own[m] += L.u[0][m][lane];
            }
#pragma unroll
            for (int m = 0; m < NDP; ++m) L.arg[odd ? kVar1[m] : kVar0[m]][pr] = own[m];
        }
        if (st > 0) {
            double Hg = H0, Sg = S0;
            for (int j = 0; j < st; ++j) {
                Hg += kR4A[st][j] * L.w[j][0][pr];
                Sg += kR4A[st][j] * L.w[j][1][pr];
            }
            s.H = Hg > 0.0 ? Hg : H0;
            s.Sh2 = Sg;
        }
        if (ok) {
            const DevParams& p = params_at(pp);
            const TConst c = load_tc(L, pr);
            const double D = L.tc[9][pr];
            ok = rhs_in<R>(p, c, arg, D, pair_inflow(a.S_in + (int64_t)s.fi * NLIQ, D, odd),
                           s.H, s.Sh2,
                           [&bv, odd](int k, double v) {
                               const int m = kVarPair[k];
                               if ((kVarSide[k] != 0) == odd) bv[m] = v;
                           },
                           s.it) == 0;
            // the first stage of the first attempt is the interval start
            if (!ok && st == 0 && s.n == 0) return 1 + 1;
            if (st == 0) {
                H0 = s.H;
                S0 = s.Sh2;
                if (ok) {
                    const DevParams& q = params_at(pp);
                    Partials d;
                    partials(q, c, arg, H0, S0, d);
                    const double alpha = ih * (1.0 / kR4Gamma);
                    {
                        const DevParams& p = q;
                        ADM1_SP2_BUILD(alpha, D);
                    }
                    ADM1_SP2_FACTOR(ok, q.pivot_floor, alpha);
                }
            }
        }
        if (ok) {
            if (st < kR4Stages - 1) {
                for (int j = 0; j < st; ++j) {
                    const double cj = kR4C[st][j] * ih;
#pragma unroll
                    for (int m = 0; m < NDP; ++m) bv[m] += cj * L.u[j][m][lane];
                }
            } else {
#pragma unroll
                for (int m = 0; m < NDP; ++m) bv[m] += ih * L.u[1][m][lane];
            }
            bv[NP - 1] = 0.0;
            ADM1_SP2_SOLVE();
            if (st < kStored) {
#pragma unroll
                for (int m = 0; m < NDP; ++m) L.u[st][m][lane] = bv[m];
            } else if (st == kR4Stages - 2) {
                // fold u_1..u_5 into the sums of the last stage
#pragma unroll
                for (int m = 0; m < NDP; ++m) {
                    double sa = 0.0, sc = 0.0;
#pragma unroll
                    for (int j = 0; j < kStored; ++j) {
                        const double uj = L.u[j][m][lane];
                        sa += kR4A[kR4Stages - 1][j] * uj;
                        sc += kR4C[kR4Stages - 1][j] * uj;
                    }
                    L.u[0][m][lane] = sa + kR4A[kR4Stages - 1][kStored] * bv[m];
                    L.u[1][m][lane] = sc + kR4C[kR4Stages - 1][kStored] * bv[m];
                }
            }
            if (st < kR4Stages - 1) L.w[st][odd ? 1 : 0][pr] = bv[NP - 1];
        }
    }
    ++s.n;
    double err = INFINITY;
    double y1[NDP];
    if (ok) {
        const DevParams& p = params_at(pp);
#pragma unroll
        for (int m = 0; m < NDP; ++m) y1[m] = s.y[m] + (L.u[0][m][lane] + bv[m]);
        double e = 0.0;
        bool fin = true;
#pragma unroll
        for (int m = 0; m < NDP; ++m) {
            const double at = odd ? p.atol[kVar1[m]] : p.atol[kVar0[m]];
            const double r = bv[m] * frcp(at + p.rtol * fmax(fabs(s.y[m]), fabs(y1[m])));
            e += r * r;
            fin = fin & isfinite(y1[m]);
        }
        e += swp(e);
        const double fo = swp(fin ? 1.0 : 0.0);
        err = sqrt(e / NY);
        ok = fin & (fo == 1.0) & isfinite(err);
    }
    const double fac = ok ? step_factor(err) : 0.2;
    double hnew = hs * fac;
    if (ok && err <= 1.0) {
        ++s.acc;
#pragma unroll
        for (int m = 0; m < NDP; ++m) s.y[m] = y1[m];
        // algebraic warm start for the next step: the stage-6 roots plus the
        // linear correction of the last stage
        const double wHl = bc0(bv[NP - 1]), wSl = bc1(bv[NP - 1]);
        const double Hn = s.H + wHl;
        s.H = Hn > 0.0 ? Hn : s.H;
        s.Sh2 = s.Sh2 + wSl;
        if (s.reject_prev && hnew > hs) hnew = hs;
        s.reject_prev = false;
        if (clip) {
            s.hlast = fmax(hnew, s.h);
            return 0 + 1;
        }
        s.t += hs;
        s.h = hnew;
    } else {
        ++s.rej;
        s.reject_prev = true;
        s.h = hnew;
        s.H = H0;
        s.Sh2 = S0;
    }
    return 0;
}

template <typename R>
__global__ void __launch_bounds__(64, 1) k_step_sparse2(StepArgs a)
{
    __shared__ Lds L;
    const int lane = threadIdx.x;
    const bool odd = lane & 1;
    const int64_t total = a.index ? (int64_t)(*a.index_count) : a.n;
    cparams_t pp = (cparams_t)a.pdev;
    PairState s;
    s.pid = -1;
    bool active = false, exhausted = false;
    int job = kNone, fin_status = 0;
    const int batch = a.service_batch > 0 ? (a.service_batch < 32 ? a.service_batch : 32)
                                          : kServiceBatch;
    for (;;) {
        // pairs waiting for service (finished particles, free pairs with work
        // left) are served together: a service pass costs the whole wave
        const bool waiting = !active && (job != kNone || !exhausted);
        const int nwait = __popcll(__ballot(waiting && !odd));
        if (nwait >= batch || !__any(active))
            service<R>(a, pp, L, s, job, fin_status, active, exhausted, odd, lane, total);
        if (__all(exhausted)) break;
        if (active) {
            const int r = attempt<R>(a, pp, L, s, odd, lane);
            if (r) {
                fin_status = r - 1;
                job = kFinish;
                active = false;
            }
        }
    }
}

__global__ void k_reset_queue(int32_t* q) { q[0] = 0; }

}  // namespace

hipError_t launch_step_sparse2(const StepArgs& a, int rate_precision, int blocks_per_cu,
                               hipStream_t s)
{
    if (a.n == 0 && !a.index) return hipSuccess;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int per_cu = blocks_per_cu > 0 ? blocks_per_cu : kWavesPerCU;
    int64_t grid = (int64_t)ncu * per_cu;
    const int64_t bound = a.index ? a.index_bound : a.n;
    const int64_t need = (bound + 31) / 32;
    if ((!a.index || bound > 0) && need < grid) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, s, a.queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rate_precision)
        hipLaunchKernelGGL(k_step_sparse2<float>, dim3((unsigned)grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(k_step_sparse2<double>, dim3((unsigned)grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace adm1
