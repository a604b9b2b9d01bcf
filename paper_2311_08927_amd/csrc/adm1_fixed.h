// Launch arguments of the fixed-step explicit scheme (sec. 2.3: synchronised
// coupling steps small enough that no step-size control is needed; sec. 4.3:
// Dt = 0.5 s as ten internal steps).  The kernel is in adm1_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adm1_devparams.h"

namespace adm1 {

struct FixedArgs {
    DevParams p;
    double* state;       // [35][ld], advanced in place
    int64_t ld, n;
    const double* T;     // K
    const double* D;     // 1/d
    const int32_t* fidx;
    const double* S_in;  // [n_feed][26]
    int64_t n_feed;
    double dt;           // coupling interval, days
    int32_t substeps;    // equal explicit steps per interval
    int32_t method;      // 0 explicit Euler, 1 classical RK4
    double* H;           // nullable: S_H+ warm start in, root out
    uint8_t* status;
    int32_t* newton;     // nullable: algebraic Newton iterations per particle
    const uint8_t* phase;      // [n] nullable: phase id per particle
    const double* phase_kin;   // [256] kinetic factor per phase id
};

hipError_t launch_fixed(const FixedArgs& a, int rate_precision, hipStream_t s);

}  // namespace adm1
