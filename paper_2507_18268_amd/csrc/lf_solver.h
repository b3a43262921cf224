// Host-side entry points shared by the solver translation units.
#pragma once

#include "lf_kernels.h"

namespace lf {

inline int32_t cell_blocks(int32_t n) { return n > 0 ? (n + kCellBlock - 1) / kCellBlock : 1; }
inline dim3 cell_grid(const lf_problem *P) { return dim3(static_cast<unsigned>(P->sp.grid)); }

enum FinMode : int { kFinMean = 0, kFinStart = 1, kFinAlpha = 2, kFinBeta = 3 };
template <int Mode>
void launch_fin(lf_problem *P, hipStream_t s);

MeshRows mesh_rows(const lf_mesh *m);
void carve_problem(Carver &cv, const lf_mesh *m, const lf_solver_opts &o, lf_problem *P);
void carve_mixed(Carver &cv, const lf_mesh *m, lf_problem *P);
lf_status launch_assemble(lf_problem *P, bool full, hipStream_t s);
lf_status launch_assemble_setup(lf_problem *P, hipStream_t s);
lf_status solve_fp64(lf_problem *P, lf_solve_stats *out);
lf_status solve_mixed(lf_problem *P, lf_solve_stats *out);
lf_status launch_amul_hook(lf_problem *P, const double *x, double *y);
lf_status check_finite_device(lf_problem *P, const double *T, bool *ok);

}  // namespace lf
