// count_ops.cpp -- operation counts of the ORACLE's right-hand side.
//
// TEST/MEASUREMENT INFRASTRUCTURE ONLY: builds adm1_oracle.c unchanged as
// C++ with its scalar `cx` replaced by a counting type, and reports how many
// arithmetic operations each part of the right-hand side takes (the
// per-evaluation flop figures of the algorithmic flop model).  The HIP path
// never loads it.
//
// Counting rules (the algorithmic count of the method, not of this code):
//   * add, subtract, multiply on a counted value: 1 each; a multiply by an
//     exact 0 or +-1 and an add of an exact 0 are not counted (structural
//     zeros and unit coefficients of the Petersen matrix: a code that knows
//     the structure skips them);
//   * divide: 1, also tallied separately;
//   * exp, log, pow, sqrt: 1 each, also tallied separately (on counted values
//     and on plain doubles alike, through the macros below);
//   * comparisons and copies: 0.
// Products of two plain parameters (loop-invariant) are not counted.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>

namespace cnt {
struct Tally {
    uint64_t add, mul, div, exp, log, pow, sqrt;
};
static Tally t;
static inline bool triv_mul(double a) { return a == 0.0 || a == 1.0 || a == -1.0; }
}  // namespace cnt

struct Counted {
    std::complex<double> z;
    Counted() : z(0.0) {}
    Counted(double v) : z(v) {}  // NOLINT: implicit, like double -> double complex
    Counted(std::complex<double> v) : z(v) {}
};
static inline double creal(const Counted& a) { return a.z.real(); }
static inline double cimag(const Counted& a) { return a.z.imag(); }
static inline double cnt_val(double a) { return a; }
static inline double cnt_val(const Counted& a) { return a.z.real(); }

template <class A, class B>
static inline Counted cnt_add(const A& a, const B& b, bool sub)
{
    const double va = cnt_val(a), vb = cnt_val(b);
    if (!(va == 0.0 || vb == 0.0)) ++cnt::t.add;
    const Counted ca(a), cb(b);
    return Counted(sub ? ca.z - cb.z : ca.z + cb.z);
}
template <class A, class B>
static inline Counted cnt_mul(const A& a, const B& b)
{
    if (!(cnt::triv_mul(cnt_val(a)) || cnt::triv_mul(cnt_val(b)))) ++cnt::t.mul;
    const Counted ca(a), cb(b);
    return Counted(ca.z * cb.z);
}
template <class A, class B>
static inline Counted cnt_div(const A& a, const B& b)
{
    ++cnt::t.div;
    const Counted ca(a), cb(b);
    return Counted(ca.z / cb.z);
}

#define CNT_OPS(T1, T2)                                                                    \
    static inline Counted operator+(const T1& a, const T2& b) { return cnt_add(a, b, false); } \
    static inline Counted operator-(const T1& a, const T2& b) { return cnt_add(a, b, true); }  \
    static inline Counted operator*(const T1& a, const T2& b) { return cnt_mul(a, b); }        \
    static inline Counted operator/(const T1& a, const T2& b) { return cnt_div(a, b); }
CNT_OPS(Counted, Counted)
CNT_OPS(Counted, double)
CNT_OPS(double, Counted)
#undef CNT_OPS
static inline Counted operator-(const Counted& a) { return Counted(-a.z); }
static inline Counted& operator+=(Counted& a, const Counted& b) { return a = a + b; }
static inline Counted& operator-=(Counted& a, const Counted& b) { return a = a - b; }
static inline Counted& operator*=(Counted& a, const Counted& b) { return a = a * b; }
static inline Counted& operator+=(Counted& a, double b) { return a = a + b; }
static inline Counted& operator-=(Counted& a, double b) { return a = a - b; }

static inline double cnt_exp(double a) { ++cnt::t.exp; return std::exp(a); }
static inline double cnt_log(double a) { ++cnt::t.log; return std::log(a); }
static inline double cnt_pow(double a, double b) { ++cnt::t.pow; return std::pow(a, b); }
static inline double cnt_sqrt(double a) { ++cnt::t.sqrt; return std::sqrt(a); }
static inline Counted cpow(const Counted& a, double b)
{
    ++cnt::t.pow;
    return Counted(std::pow(a.z, b));
}
static const Counted I(std::complex<double>(0.0, 1.0));

#define ORC_COUNTED 1
typedef Counted cx;
#define exp(x) cnt_exp(x)
#define log(x) cnt_log(x)
#define pow(a, b) cnt_pow(a, b)
#define sqrt(x) cnt_sqrt(x)
#include "adm1_oracle.c"
#undef exp
#undef log
#undef pow
#undef sqrt

namespace {
void take(double* out)
{
    out[0] = (double)cnt::t.add;
    out[1] = (double)cnt::t.mul;
    out[2] = (double)cnt::t.div;
    out[3] = (double)cnt::t.exp;
    out[4] = (double)cnt::t.log;
    out[5] = (double)cnt::t.pow;
    out[6] = (double)cnt::t.sqrt;
    std::memset(&cnt::t, 0, sizeof(cnt::t));
}
}  // namespace

// Counts for one particle state x[35] at temperature T, dilution D, inflow
// s_in[26].  out: 7 parts x 7 tallies (add, mul, div, exp, log, pow, sqrt):
//   0 temperature constants, 1 rates and transfers at the solved roots (one
//   call of rates()), 2 the eq.-2 assembly and headspace balances (rhs()
//   without its algebraic solves and rates), 3 one eq.-7 residual with its
//   derivative, 4 one eq.-8 residual with its derivative, 5 the algebraic
//   write-back of the six ions, 6 one whole rhs() including its bracketed
//   solves.  Returns the eq.-7 and eq.-8 Newton iterations of that rhs() in
//   iters[0].
extern "C" int orc_count_rhs(const orc_params* p, const orc_opts* o, const double* x,
                             double T, double D, const double* s_in, double* out,
                             int* iters)
{
    std::memset(&cnt::t, 0, sizeof(cnt::t));
    orc_model m;
    m.p = p; m.o = o; m.c = orc_tconsts(p, T); m.D = D;
    take(out + 0);
    petersen(p, m.nu);
    for (int i = 0; i < NLIQ; i++) m.s_in[i] = s_in[i];
    m.H_guess = -1.0;
    m.Sh2_guess = x[S_H2];
    m.newton_iters = 0;
    cx y[ND], xa[NX], f[ND], H;
    for (int k = 0; k < ND; k++) y[k] = x[DIFF[k]];
    // converged roots first (uncounted), then each part on its own
    std::memset(&cnt::t, 0, sizeof(cnt::t));
    if (algebraic(&m, y, xa, &H)) return -1;
    std::memset(&cnt::t, 0, sizeof(cnt::t));
    orc_rates_t r;
    rates(p, &m.c, xa, H, &r);
    take(out + 7);
    // rhs() = algebraic() + rates() + assembly: count rhs and algebraic from
    // the same warm starts, subtract both
    const double Hg = m.H_guess, Sg = m.Sh2_guess;
    m.newton_iters = 0;
    if (rhs(&m, y, f, NULL)) return -1;
    double whole[7];
    take(whole);
    *iters = m.newton_iters;
    m.H_guess = Hg;
    m.Sh2_guess = Sg;
    cx xb[NX], Hb;
    if (algebraic(&m, y, xb, &Hb)) return -1;
    double alg[7];
    take(alg);
    for (int k = 0; k < 7; k++) out[14 + k] = whole[k] - alg[k] - out[7 + k];
    cx dE;
    charge_balance(p, &m.c, xa, H, &dE);
    take(out + 21);
    h2_balance(p, &m.c, xa, H, D, s_in[S_H2], m.nu, &dE);
    take(out + 28);
    // ion write-back as in algebraic()
    {
        cx w[6];
        w[0] = p->K_a_va * xa[S_VA] / (p->K_a_va + H);
        w[1] = p->K_a_bu * xa[S_BU] / (p->K_a_bu + H);
        w[2] = p->K_a_pro * xa[S_PRO] / (p->K_a_pro + H);
        w[3] = p->K_a_ac * xa[S_AC] / (p->K_a_ac + H);
        w[4] = m.c.K_a_co2 * xa[S_IC] / (m.c.K_a_co2 + H);
        w[5] = m.c.K_a_IN * xa[S_IN] / (m.c.K_a_IN + H);
        (void)w;
    }
    take(out + 35);
    for (int k = 0; k < 7; k++) out[42 + k] = whole[k];
    return 0;
}
