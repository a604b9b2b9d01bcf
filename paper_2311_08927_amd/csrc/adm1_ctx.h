// The library context behind the opaque adm1_ctx handle, and the argument
// checks shared by the entry points (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adm1.h"
#include "adm1_devparams.h"

struct adm1_ctx {
    adm1::DevParams dp;
    adm1_params raw;     // parameters as given (the surrogate gate derives from them)
    adm1_opts opts;
    int64_t n_max;
    int device;
    int32_t* d_queue;    // work-queue counter
    double* d_partial;   // gas-flux block partials [kGasBlocks][4]
    adm1::DevParams* d_params;  // device copy of dp
    int tuned_variant;   // step variant chosen by adm1_set_launch (-1: none)
    int tuned_blocks_per_cu;
    int tuned_service_batch;  // pairs served together by the persistent kernel (0: default)
    int order_mode;      // ADM1_ORDER_* of the step kernel's work queue
    int32_t* d_order;    // cost-ordered particle list [max(n_max, 1)]
    int32_t* d_order_work;  // its histogram, bucket cursors and length
    unsigned long long* d_fail;  // per-block outcome counts of the last step call [kCountBlocks][kFailSlots]
    int32_t* static_scratch;     // this device's address of the library's static scratch
    double* d_phase_kin;  // kinetic factor of each phase id [ADM1_MAX_PHASES]
};

// A captured coupling step (adm1_graph_capture_step and its surrogate
// counterpart).
struct adm1_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace adm1_abi {
bool is_device(const void* ptr);
int check_layout(const adm1_ctx* ctx, int64_t ld, int64_t n);
int check_feed(const adm1_feed* feed);
// check_feed, and no phases (calls that do not model them)
int check_feed_no_phase(const adm1_feed* feed);
int hip_rc(hipError_t e);
// End a capture begun on s, instantiate the graph into *g (freed on error).
int finish_capture(hipStream_t s, int rc, adm1_graph* g, adm1_graph** out);
}  // namespace adm1_abi
