// Kernel argument blocks and launchers of the ADM1 step (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adm1_devparams.h"

namespace adm1 {

struct StepArgs {
    DevParams p;
    double* state;          // [35][ld]
    int64_t ld, n;
    const double* T;        // [n]
    const double* D;        // [n]
    const int32_t* fidx;    // [n]
    const double* S_in;     // [n_feed][26]
    int64_t n_feed;
    double dt;
    double* H;              // [n] nullable
    double* hlast;          // [n] nullable
    uint8_t* status;        // [n]
    int32_t* nsteps;        // [3][ld] nullable
    int32_t* queue;         // work-queue counter (persistent kernels)
    const int32_t* index;   // optional particle index list (nullable: identity)
    const int32_t* index_count;  // device count of the index list (with index)
    int64_t index_bound;    // host upper bound of that count (0: unknown)
    const DevParams* pdev;  // device copy of p (read through the scalar cache)
    int32_t service_batch;  // persistent kernel: pairs served together (0: default)
    const uint8_t* phase;      // [n] nullable: phase id per particle
    const double* phase_kin;   // [256] kinetic factor per phase id
};

struct RhsArgs {
    DevParams p;
    const double* state;
    int64_t ld, n;
    const double* T;
    const double* D;
    const int32_t* fidx;
    const double* S_in;
    int64_t n_feed;
    double* dxdt;
    int64_t ld_out;
    double* H_out;
    uint8_t* status;
    const uint8_t* phase;      // [n] nullable: phase id per particle
    const double* phase_kin;   // [256] kinetic factor per phase id
};

struct GasArgs {
    DevParams p;
    const double* state;
    int64_t ld, n, chunk;
    const double* T;
    const double* V_liq;
    double* q_gas;
    double* q_ch4;
    double* partial;  // [nblocks][4]
};

// One lane per particle; lin: 0 dense pivoted LU (private memory), 1 static
// sparse LU in registers, 2 static sparse LU with the matrix in LDS.
hipError_t launch_step1(const StepArgs& a, int rate_precision, int lin, hipStream_t s);
hipError_t launch_step_sparse2(const StepArgs& a, int rate_precision, int blocks_per_cu,
                               hipStream_t s);
// Cost order of the work queue: order[0..len-1] = particles by non-increasing
// bucket min(floor(kOrderRes dt / hlast[i]), kOrderBuckets-1) (the last
// bucket also for hlast[i] <= 0 or NaN).  Without a list the particles are
// 0..n-1 (len = n); with one they are list[0..len-1], len = min(*list_count,
// n) read on the device (n is then the list's capacity).  work: int32
// [2 kOrderBuckets + 1], zero in its first kOrderBuckets entries before the
// first call (left so); work[2 kOrderBuckets] receives len for the queue.
constexpr int kOrderBuckets = 1024;
constexpr double kOrderRes = 8.0;
hipError_t launch_cost_order(const double* hlast, const int32_t* list,
                             const int32_t* list_count, int64_t n, double dt, int32_t* work,
                             int32_t* order, hipStream_t s);
struct PhArgs {
    DevParams p;
    const double* state;    // [35][ld]
    int64_t ld, n;
    const double* T;        // [n]
    const double* guess;    // [n] nullable
    double* H_out;          // [n]
    double* pH_out;         // [n] nullable
    uint8_t* status;        // [n] nullable
};

// Outcome counters of the last step call on a context (adm1_last_failures):
// [0] particles with a nonzero status code, [1..4] codes 1..4, [5] code 0
// with the negative-entry bit, [6] particles counted.
constexpr int kFailSlots = 7;

hipError_t launch_rhs(const RhsArgs& a, int rate_precision, hipStream_t s);
hipError_t launch_solve_ph(const PhArgs& a, hipStream_t s);
hipError_t launch_count_status(const uint8_t* status, int64_t n, unsigned long long* counts,
                               hipStream_t s);
hipError_t launch_jacobian(const RhsArgs& a, double* J, hipStream_t s);
hipError_t launch_gasflux(const GasArgs& a, int nblocks, double* totals, hipStream_t s);

}  // namespace adm1
