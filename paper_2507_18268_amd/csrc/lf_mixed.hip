// Mixed-precision iterative refinement (FP64 outer, FP32 inner PCG).
#include <hip/hip_runtime.h>

#include "lf_kernels.h"

using namespace lf;

lf_status lf_solve_mixed(lf_problem *P, lf_solve_stats *out) {
    (void)P;
    (void)out;
    set_error("mixed precision not built yet");
    return LF_EINVAL;
}
