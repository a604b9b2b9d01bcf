// Two-lanes-per-particle step (register-resident sparse LU).
#include <hip/hip_runtime.h>

#include "adm1_kernels.h"

namespace adm1 {

hipError_t launch_step_sparse2(const StepArgs&, int, int, hipStream_t)
{
    return hipErrorInvalidDeviceFunction;
}

}  // namespace adm1
