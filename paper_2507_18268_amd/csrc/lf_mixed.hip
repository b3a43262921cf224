// Mixed-precision iterative refinement (FP64 outer, FP32 inner PCG).
#include <hip/hip_runtime.h>

#include "lf_solver.h"

namespace lf {

void carve_mixed(Carver &cv, const lf_mesh *m, lf_problem *P) {
    const size_t N = m->N;
    auto *coef32 = cv.take<float>(static_cast<size_t>(m->n_entries));
    float *v32[6];
    for (auto &v : v32) v = cv.take<float>(N);
    auto *tsave = cv.take<double>(N);
    if (P) {
        P->coef32 = coef32; P->diag32 = v32[0]; P->rD32 = v32[1]; P->r32 = v32[2];
        P->p32 = v32[3]; P->q32 = v32[4]; P->d32 = v32[5]; P->Tsave = tsave;
    }
}

lf_status solve_mixed(lf_problem *P, lf_solve_stats *out) {
    (void)P;
    (void)out;
    set_error("mixed precision not built yet");
    return LF_EINVAL;
}

}  // namespace lf
