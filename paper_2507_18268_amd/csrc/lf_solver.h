// Host-side entry points shared by the solver translation units.
#pragma once

#include "lf_kernels.h"

namespace lf {

inline int32_t cell_blocks(int32_t n) { return n > 0 ? (n + kCellBlock - 1) / kCellBlock : 1; }
inline dim3 cell_grid(const lf_problem *P) { return dim3(static_cast<unsigned>(P->sp.grid)); }
inline int32_t mx_blocks(int32_t n) {
    constexpr int32_t kTile = kCellBlock * kMxRows;
    return n > 0 ? (n + kTile - 1) / kTile : 1;
}
inline dim3 mx_grid(const lf_problem *P) { return dim3(static_cast<unsigned>(P->sp.grid_mx)); }
// workgroups of the FP64 update with the diagonal preconditioner
inline int32_t update_blocks(int32_t n) {
    constexpr int32_t kTile = kCellBlock * kUpdRows;
    return n > 0 ? (n + kTile - 1) / kTile : 1;
}

enum FinMode : int { kFinMean = 0, kFinStart = 1, kFinAlpha = 2, kFinBeta = 3, kFinConv = 4, kFinBetaOnly = 5 };
template <int Mode>
void launch_fin(lf_problem *P, hipStream_t s);

MeshRows mesh_rows(const lf_mesh *m);

// Which coefficient layout a problem uses: the band layout for the diagonal
// preconditioner on a mesh with band form, the two-colour band layout for DIC
// on a mesh with that form (LF_LAYOUT_BANDS asks for one of them;
// lf_problem_create checks that it applies), else the sliced rows.
inline bool use_bands(const lf_mesh *m, const lf_solver_opts &o) {
    if (o.layout == LF_LAYOUT_ROWS || m->n_bands == 0 || o.precond == LF_PC_DIC) return false;
    return true;
}
inline bool use_rb(const lf_mesh *m, const lf_solver_opts &o) {
    return o.layout != LF_LAYOUT_ROWS && m->rb_h > 0 && o.precond == LF_PC_DIC;
}
// coefficient slots of a problem's layout
inline size_t coef_slots(const lf_mesh *m, bool banded, bool rb = false) {
    if (rb) return 6 * static_cast<size_t>(m->n_red);
    return banded ? static_cast<size_t>(m->n_bands) * m->N : static_cast<size_t>(m->n_entries);
}

inline RBForm rb_form(const lf_mesh *m) { return RBForm{m->n_red, m->rb_h, m->rb_H, m->rb_ny}; }
inline RBLayout rb_layout(const lf_mesh *m) { return RBLayout{rb_form(m), m->rb_mag_sf, m->rb_delta}; }

inline SellLayout sell_layout(const lf_mesh *m) {
    return SellLayout{mesh_rows(m), m->mag_sf, m->delta, m->emag_sf, m->edelta};
}

template <int K>
inline BandLayout<K> band_layout(const lf_mesh *m) {
    BandLayout<K> L;
    L.n = m->N;
    for (int k = 0; k < K; ++k) L.d[k] = m->band_d[k];
    L.mag_sf = m->band_mag_sf;
    L.delta = m->band_delta;
    return L;
}

// Calls fn(layout) with the problem's layout object (a kernel template
// argument is then decltype(layout)).
template <class Fn>
inline void with_layout(const lf_problem *P, Fn &&fn) {
    const lf_mesh *m = P->mesh;
    if (P->rb) {
        fn(rb_layout(m));
        return;
    }
    if (!P->banded) {
        fn(sell_layout(m));
        return;
    }
    switch (m->n_bands) {
        case 1: fn(band_layout<1>(m)); break;
        case 2: fn(band_layout<2>(m)); break;
        case 3: fn(band_layout<3>(m)); break;
        default: fn(band_layout<4>(m)); break;
    }
}
void carve_problem(Carver &cv, const lf_mesh *m, const lf_solver_opts &o, lf_problem *P);
// multigrid preconditioner (lf_amg.hip): work space, coarse matrices (after
// each assembly), one cycle w = M r with the w.r partials
void carve_amg(Carver &cv, const lf_mesh *m, lf_problem *P);
void launch_amg_galerkin(lf_problem *P, hipStream_t s);
void launch_amg_cycle(lf_problem *P, hipStream_t s);
void carve_mixed(Carver &cv, const lf_mesh *m, bool banded, lf_problem *P);
lf_status launch_assemble(lf_problem *P, bool full, hipStream_t s);
lf_status launch_assemble_setup(lf_problem *P, hipStream_t s);
// precision form: FP32 coefficients of the scaled matrix, after the assembly
void launch_mx_scale(lf_problem *P, hipStream_t s);
lf_status launch_amul_inner_hook(lf_problem *P, const float *x, float *y);
// groups (lf_group.hip): inner iterations of several problems per launch
MemberDesc member_desc(const lf_problem *P);
// launches over the members of gl (cells: each member's sp.grid workgroups;
// inner: its sp.grid_mx; finalize: one per member)
void launch_group_setup(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s);
void launch_group_scale(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s);
void launch_group_fin_start(const MemberDesc *tab, const GroupLaunch &gl, hipStream_t s);
void launch_group_pass_start(const MemberDesc *tab, const GroupLaunch &gl, hipStream_t s);
void launch_group_pass_end(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s);
void launch_group_iteration(const MemberDesc *tab, const GroupLaunch &inner, hipStream_t s);
void launch_group_gather(const MemberDesc *tab, const GroupLaunch &gl, PcgState *out, hipStream_t s);
// non-orthogonal meshes: boundary values and gradient of T, then (correction:
// on band meshes the assembly can form it instead) P->lap_src (lf_grad.hip);
// runs before the assembly of each step
void launch_nonorth_source(lf_problem *P, hipStream_t s, bool correction = true);
lf_status launch_problem_grad(lf_problem *P, double *grad, double *bgrad);
// A solve is driven in two halves so that one host loop can drive several
// problems on their own streams: *_start enqueues the set-up and the first
// block of iterations, followed by an async copy of the solver state and
// P->ev[2]; once that event has completed, *_advance reads the state and
// either enqueues the next block (again ending with the copy and ev[2]) or
// reports the solve finished, its stats in *out.
struct SolveCtx {
    int32_t fixed_k = 0;   // iterations per block when fixed (>0), else adaptive
    int32_t k = 0;         // iterations of the next block
    int32_t launched = 0;  // iterations enqueued so far
    int32_t stage = 0;     // FP64: 0 iterating, 1 committing; mixed: 1 awaiting the
                           // outer check of a pass before starting another
};
lf_status fp64_start(lf_problem *P, SolveCtx &c);
lf_status fp64_advance(lf_problem *P, SolveCtx &c, bool *finished, lf_solve_stats *out);
lf_status mixed_start(lf_problem *P, SolveCtx &c);
lf_status mixed_advance(lf_problem *P, SolveCtx &c, bool *finished, lf_solve_stats *out);
lf_status launch_amul_hook(lf_problem *P, const double *x, double *y);
lf_status launch_precondition_hook(lf_problem *P);
lf_status check_finite_device(lf_problem *P, const double *T, bool *ok);

}  // namespace lf
