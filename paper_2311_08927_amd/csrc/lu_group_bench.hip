// Lanes per particle for the register-resident sparse LU of the bordered
// Newton matrix (sec. 2.2, eqs. 7-8 bordering the eq.-2 rows): the same
// static-order factorisation and six forward / backward substitutions (one
// per Rodas4 stage, each right-hand side depending on the previous
// solution, as the stages do) with the rows of a particle spread over G = 2
// or G = 4 lanes.  Matrices are seeded and diagonally dominant on the
// structural pattern of the step kernel's matrix; results are checked
// against a dense host solve.  Standalone measurement program, not part of
// the library.
//
// usage: lu_group_bench [n_particles (default 2^18)] [repeats]
// prints one JSON line per G with the kernel time of the full sequence, of
// the matrix set-up alone, registers and scratch per lane, and the largest
// relative error against the host solve over the checked particles.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                     \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            std::fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

constexpr int NV = 30;

__host__ __device__ inline uint32_t fmix(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
// uniform in [-1, 1) from (particle, row, column)
__host__ __device__ inline double hval(uint32_t pid, int r, int c)
{
    const uint32_t h = fmix(pid * 0x9E3779B1u ^ fmix((uint32_t)(r * 131 + c * 7 + 1)));
    return (double)(h >> 8) * (2.0 / 16777216.0) - 1.0;
}
__host__ __device__ inline double entry(uint32_t pid, int r, int c)
{
    return (r == c ? 40.0 : 0.0) + hval(pid, r, c);
}
__host__ __device__ inline double rhsv(uint32_t pid, int r, int s)
{
    return hval(pid + 7777u * (uint32_t)(s + 1), r, 101);
}
constexpr double kTheta = 0.25;  // b_{s+1} = rhs_{s+1} + theta x_s

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

#define LUG_KERNEL_BODY                                                              \
    const int lane = threadIdx.x;                                                    \
    const int sd = lane & (LUG_G - 1);                                               \
    int64_t p64 = ((int64_t)blockIdx.x * 64 + lane) / LUG_G;                         \
    const bool live = p64 < n;                                                       \
    if (!live) p64 = n - 1; /* every lane takes part in the broadcasts */           \
    const uint32_t pid = (uint32_t)p64;                                              \
    LUG_DECL;                                                                        \
    LUG_ROWVARS;                                                                     \
    LUG_INIT(ENTRY_OF);                                                              \
    if (mode == 0) {                                                                 \
        double acc = 0.0;                                                            \
        LUG_SUM(acc);                                                                \
        if (live && sd == 0) out[p64 * NV] = acc;                                    \
        return;                                                                      \
    }                                                                                \
    bool ok = true;                                                                  \
    LUG_FACTOR(ok);                                                                  \
    LUG_BSET(RHS0);                                                                  \
    _Pragma("unroll 1") for (int s = 0; s < 6; ++s) {                              \
        if (s > 0) { LUG_BNEXT(RHSS, kTheta); }                                      \
        LUG_SOLVE();                                                                 \
    }                                                                                \
    if (live) { LUG_STORE(STORE_TO); }                                               \
    if (!ok && live) out[p64 * NV] = NAN;

#define ENTRY_OF(r, c) A[(size_t)((r) * NV + (c)) * (size_t)n + pid]
#define RHS0(r) rhsv(pid, r, 0)
#define RHSS(r) rhsv(pid, r, s)
#define STORE_TO(r, v) out[p64 * NV + (r)] = (v)

namespace g2 {
template <int S>
__device__ __forceinline__ double bcast(double v)
{
    return dpp<S == 0 ? 0xA0 : 0xF5>(v);  // quad_perm [0,0,2,2] / [1,1,3,3]
}
#include <lu_g2.inc>
__global__ void __launch_bounds__(64, 1) k_lu(int64_t n, int mode, const double* __restrict__ A,
                                             double* out)
{
    LUG_KERNEL_BODY
}
}  // namespace g2
#undef LUG_G
#undef LUG_NGROUP
#undef LUG_DECL
#undef LUG_ROWVARS
#undef LUG_INIT
#undef LUG_BSET
#undef LUG_BNEXT
#undef LUG_STORE
#undef LUG_SUM
#undef LUG_NSTRUCT
#undef LUG_STRUCT
#undef LUG_FACTOR
#undef LUG_SOLVE

namespace g4 {
template <int S>
__device__ __forceinline__ double bcast(double v)
{
    return dpp<S * 0x55>(v);  // quad_perm [S,S,S,S]
}
#include <lu_g4.inc>
__global__ void __launch_bounds__(64, 1) k_lu(int64_t n, int mode, const double* __restrict__ A,
                                             double* out)
{
    LUG_KERNEL_BODY
}
constexpr int kStruct[LUG_NSTRUCT][2] = LUG_STRUCT;
}  // namespace g4

// dense host solve of particle pid's sequence (partial pivoting)
static void host_sequence(uint32_t pid, double* x)
{
    double A[NV][NV] = {};
    for (const auto& e : g4::kStruct) A[e[0]][e[1]] = entry(pid, e[0], e[1]);
    int perm[NV];
    for (int i = 0; i < NV; ++i) perm[i] = i;
    for (int k = 0; k < NV; ++k) {
        int p = k;
        for (int i = k + 1; i < NV; ++i)
            if (std::fabs(A[i][k]) > std::fabs(A[p][k])) p = i;
        if (p != k) {
            for (int j = 0; j < NV; ++j) std::swap(A[k][j], A[p][j]);
            std::swap(perm[k], perm[p]);
        }
        for (int i = k + 1; i < NV; ++i) {
            const double l = A[i][k] / A[k][k];
            A[i][k] = l;
            for (int j = k + 1; j < NV; ++j) A[i][j] -= l * A[k][j];
        }
    }
    double prev[NV] = {};
    for (int s = 0; s < 6; ++s) {
        double b[NV], y[NV];
        for (int i = 0; i < NV; ++i) b[i] = rhsv(pid, i, s) + (s > 0 ? kTheta * prev[i] : 0.0);
        for (int i = 0; i < NV; ++i) {
            double v = b[perm[i]];
            for (int j = 0; j < i; ++j) v -= A[i][j] * y[j];
            y[i] = v;
        }
        for (int i = NV - 1; i >= 0; --i) {
            double v = y[i];
            for (int j = i + 1; j < NV; ++j) v -= A[i][j] * prev[j];
            prev[i] = v / A[i][i];
        }
    }
    for (int i = 0; i < NV; ++i) x[i] = prev[i];
}

template <int G>
static void run(void (*kern)(int64_t, int, const double*, double*), const char* name, int64_t n,
                int reps, const double* d_A)
{
    double* d_out;
    CHECK(hipMalloc(&d_out, (size_t)n * NV * sizeof(double)));
    const int64_t lanes = n * G;
    const dim3 grid((unsigned)((lanes + 63) / 64)), block(64);
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    float best[2] = {1e30f, 1e30f};
    for (int mode = 0; mode < 2; ++mode) {
        for (int r = 0; r < reps + 1; ++r) {
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(kern, grid, block, 0, 0, n, mode, d_A, d_out);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, a, b));
            if (r > 0 && ms < best[mode]) best[mode] = ms;  // first run warms up
        }
    }
    // check the last (mode 1) results of the first and last particles
    const int nchk = 64;
    std::vector<double> got((size_t)nchk * NV), want(NV);
    double worst = 0.0;
    for (int part = 0; part < 2; ++part) {
        const int64_t p0 = part == 0 ? 0 : n - nchk;
        CHECK(hipMemcpy(got.data(), d_out + p0 * NV, got.size() * sizeof(double),
                        hipMemcpyDeviceToHost));
        for (int q = 0; q < nchk; ++q) {
            host_sequence((uint32_t)(p0 + q), want.data());
            double scale = 0.0;
            for (int i = 0; i < NV; ++i) scale = std::fmax(scale, std::fabs(want[i]));
            for (int i = 0; i < NV; ++i)
                worst = std::fmax(worst, std::fabs(got[(size_t)q * NV + i] - want[i]) / scale);
        }
    }
    hipFuncAttributes fa;
    CHECK(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
    std::printf("{\"lanes_per_particle\": %d, \"kernel\": \"%s\", \"particles\": %lld, "
                "\"ms_factor_6solves\": %.4f, \"ms_setup_only\": %.4f, "
                "\"ns_per_particle_lu\": %.4f, \"vgpr\": %d, \"scratch_bytes_per_lane\": %zu, "
                "\"max_rel_err\": %.3e}\n",
                G, name, (long long)n, best[1], best[0],
                1e6 * (best[1] - best[0]) / (double)n, fa.numRegs, fa.localSizeBytes, worst);
    std::fflush(stdout);
    CHECK(hipFree(d_out));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
}

int main(int argc, char** argv)
{
    const int64_t n = argc > 1 ? std::atoll(argv[1]) : (1 << 18);
    const int reps = argc > 2 ? std::atoi(argv[2]) : 5;
    if (n < 64 || n > (1 << 22) || reps < 1) {
        std::fprintf(stderr, "need 64 <= n <= 2^22 and repeats >= 1\n");
        return 2;
    }
    // the matrices, structure-of-arrays A[row * 30 + col][particle]; only the
    // structural entries are read
    std::vector<double> hA((size_t)NV * NV * n, 0.0);
    for (const auto& e : g4::kStruct)
        for (int64_t q = 0; q < n; ++q)
            hA[(size_t)(e[0] * NV + e[1]) * n + q] = entry((uint32_t)q, e[0], e[1]);
    double* d_A;
    CHECK(hipMalloc(&d_A, hA.size() * sizeof(double)));
    CHECK(hipMemcpy(d_A, hA.data(), hA.size() * sizeof(double), hipMemcpyHostToDevice));
    run<2>(g2::k_lu, "g2", n, reps, d_A);
    run<4>(g4::k_lu, "g4", n, reps, d_A);
    CHECK(hipFree(d_A));
    return 0;
}
