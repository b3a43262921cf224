// C interface of the problem handle (see include/lapfoam.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "lf_solver.h"

using namespace lf;

// One problem's stepping: lf_step and lf_step_many run it to the end;
// lf_step_begin keeps one in the problem and lf_step_poll advances it.
namespace lf {
struct StepDriver {
    lf_problem *P = nullptr;
    lf_solve_stats *stats = nullptr;   // [n_steps] or null
    double *snap = nullptr;            // device [n_steps][N], mesh order, or null
    int32_t n_steps = 0, step = 0;
    SolveCtx c;
    lf_solve_stats cur{};
    int32_t pass = 0;                  // pass of the non-orthogonal corrector loop
    lf_solve_stats acc{};              // the step's earlier passes
    bool active = false, nonfinite = false;
    std::vector<lf_solve_stats> own_stats;   // lf_step_begin's stats
};
}  // namespace lf

namespace lf {
bool problem_in_flight(const lf_problem *P) { return (P->async && P->async->active) || P->group; }
}  // namespace lf

static bool async_running(const lf_problem *P) { return problem_in_flight(P); }

extern "C" {

lf_status lf_default_opts(lf_solver_opts *o) {
    if (!o) return LF_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-9;
    o->rel_tol = 0.0;
    o->max_iter = 1000;
    o->min_iter = 0;
    o->precond = LF_PC_DIAGONAL;
    o->precision = LF_PREC_FP64;
    o->iters_per_check = 0;
    o->use_graph = 1;
    o->inner_tol = 0.0;
    o->max_outer = 0;
    o->layout = LF_LAYOUT_AUTO;
    o->amul_walk = LF_WALK_AUTO;
    o->inner_restart = 0;
    o->n_nonorth_corr = 0;
    return LF_OK;
}

size_t lf_problem_workspace_bytes(const lf_mesh *m, const lf_solver_opts *o) {
    if (!m) return 0;
    lf_solver_opts d;
    lf_default_opts(&d);
    Carver cv(nullptr);
    carve_problem(cv, m, o ? *o : d, nullptr);
    return cv.bytes();
}

// boundary conditions, DT and dt of a problem on mesh m
static lf_status check_physics(const lf_mesh *m, const lf_patch_bc *bcs, double DT, double dt) {
    if (m->P > 0 && !bcs) { set_error("bcs is NULL"); return LF_EINVAL; }
    if (!(DT >= 0.0) || !std::isfinite(DT)) { set_error("DT must be finite and >= 0"); return LF_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be finite and > 0"); return LF_EINVAL; }
    for (int32_t p = 0; p < m->P; ++p) {
        if (bcs[p].type != LF_BC_ZERO_GRADIENT && bcs[p].type != LF_BC_FIXED_VALUE) {
            set_error("patch %d: unknown boundary condition type %d", p, bcs[p].type);
            return LF_EINVAL;
        }
        if (bcs[p].type == LF_BC_FIXED_VALUE && !std::isfinite(bcs[p].value)) {
            set_error("patch %d: fixed value not finite", p);
            return LF_EINVAL;
        }
    }
    return LF_OK;
}

lf_status lf_problem_create(const lf_mesh *m, const lf_patch_bc *bcs, double DT, double dt,
                            const lf_solver_opts *o, void *ws, size_t ws_bytes, void *stream, lf_problem **out) {
    clear_error();
    if (!out) { set_error("out is NULL"); return LF_EINVAL; }
    *out = nullptr;
    if (!m) { set_error("mesh is NULL"); return LF_EINVAL; }
    if (!m->orthogonal && !m->gkband && !m->gkerec) {
        set_error("a mesh with non-orthogonal faces needs face centres (the correction's gradient)");
        return LF_EINVAL;
    }
    LF_TRY(check_physics(m, bcs, DT, dt));
    lf_solver_opts opts;
    if (o) opts = *o; else lf_default_opts(&opts);
    if (opts.max_iter < 0 || opts.min_iter < 0 || !std::isfinite(opts.tol) || !std::isfinite(opts.rel_tol) ||
        !std::isfinite(opts.inner_tol) || opts.inner_tol < 0.0 || opts.inner_tol >= 1.0 || opts.max_outer < 0 ||
        opts.n_nonorth_corr < 0 || opts.n_nonorth_corr > 100) {
        set_error("bad solver options");
        return LF_EINVAL;
    }
    if (opts.precond != LF_PC_DIAGONAL && opts.precond != LF_PC_DIC && opts.precond != LF_PC_AMG) {
        set_error("unknown preconditioner");
        return LF_EINVAL;
    }
    if (opts.precond == LF_PC_AMG && (m->box_nx == 0 || opts.layout == LF_LAYOUT_ROWS)) {
        set_error("the multigrid preconditioner needs a box mesh numbered i + nx (j + ny k) (band offsets 1, nx, "
                  "nx ny, sides >= 2) and the band layout");
        return LF_EINVAL;
    }
    if (opts.precond == LF_PC_AMG && opts.precision == LF_PREC_MIXED) {
        set_error("the mixed-precision form uses the diagonal preconditioner");
        return LF_EINVAL;
    }
    if (opts.precision != LF_PREC_FP64 && opts.precision != LF_PREC_MIXED) { set_error("unknown precision"); return LF_EINVAL; }
    if (opts.precond == LF_PC_DIC && m->F > 0 && !m->two_colour) {
        set_error("DIC needs a two-colour numbering (every owner < every neighbour)");
        return LF_EINVAL;
    }
    if (opts.layout != LF_LAYOUT_AUTO && opts.layout != LF_LAYOUT_ROWS && opts.layout != LF_LAYOUT_BANDS) {
        set_error("unknown layout %d", opts.layout);
        return LF_EINVAL;
    }
    if (opts.inner_restart != 0 && opts.inner_restart != 1) {
        set_error("inner_restart must be 0 or 1");
        return LF_EINVAL;
    }
    if (opts.amul_walk != LF_WALK_AUTO && opts.amul_walk != LF_WALK_ON && opts.amul_walk != LF_WALK_OFF) {
        set_error("unknown amul_walk %d", opts.amul_walk);
        return LF_EINVAL;
    }
    if (opts.layout == LF_LAYOUT_BANDS && opts.precond == LF_PC_DIAGONAL && m->n_bands == 0) {
        set_error("the band layout needs a mesh whose faces take at most %d offsets", kMaxBands);
        return LF_EINVAL;
    }
    if (opts.layout == LF_LAYOUT_BANDS && opts.precond == LF_PC_DIC && m->rb_h == 0) {
        set_error("the band layout with DIC needs a two-colour numbered box whose x-lines hold an even "
                  "number of cells");
        return LF_EINVAL;
    }
    if (opts.precond == LF_PC_DIC && opts.precision == LF_PREC_MIXED) {
        set_error("the mixed-precision form uses the diagonal preconditioner");
        return LF_EINVAL;
    }
    Carver dry(nullptr);
    carve_problem(dry, m, opts, nullptr);
    if (!ws || ws_bytes < dry.bytes() || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
        set_error("problem workspace too small or misaligned: need %zu bytes, 256-aligned", dry.bytes());
        return LF_ENOMEM;
    }
    int dev = 0;
    LF_HIP(hipGetDevice(&dev));
    if (dev != m->device) { set_error("problem created on device %d, mesh on %d", dev, m->device); return LF_EINVAL; }
    lf_problem *P = new (std::nothrow) lf_problem();
    if (!P) { set_error("host allocation failed"); return LF_ENOMEM; }
    P->mesh = m;
    P->opts = opts;
    P->DT = DT;
    P->dt = dt;
    P->stream = static_cast<hipStream_t>(stream);
    P->banded = use_bands(m, opts);
    P->rb = use_rb(m, opts);
    P->nonorth = !m->orthogonal;
    P->sp.tol = opts.tol;
    P->sp.rel_tol = opts.rel_tol;
    P->sp.max_iter = opts.max_iter;
    P->sp.min_iter = opts.min_iter;
    P->sp.n = m->N;
    P->sp.grid = cell_blocks(m->N);
    P->sp.grid_mx = mx_blocks(m->N);
    P->sp.grid_upd = opts.precond == LF_PC_DIAGONAL ? update_blocks(m->N) : P->sp.grid;
    P->sp.grid_amul = P->sp.grid;
    P->sp.grid_mx_amul = P->sp.grid_mx;
    if (P->banded && m->n_bands >= 2 && opts.amul_walk != LF_WALK_OFF) {
        // the walk's partials must fit the p.q slot of both solvers' reductions
        const int32_t wb = walk_blocks(m->N, m->band_d[1]);
        BoxWalk bw, bw32;
        const bool box_plan = box_walk_plan(m->N, m->n_bands, m->band_d, 2, &bw);
        if ((opts.amul_walk == LF_WALK_ON || wb >= kWalkMinBlocks || (box_plan && bw.blocks >= kBoxMinBlocks)) &&
            wb <= P->sp.grid_mx) {
            P->walk = true;
            P->sp.grid_amul = wb;
            P->sp.grid_mx_amul = wb;
        }
        // the products of a box take the block walk: two FP64 rows or four
        // FP32 rows per lane (its partials must fit the same slots)
        if (P->walk && box_plan && bw.blocks <= P->sp.grid_mx && bw.blocks <= P->sp.grid) {
            P->box = true;
            P->bw = bw;
            P->sp.grid_amul = bw.blocks;
            if (box_walk_plan(m->N, m->n_bands, m->band_d, 4, &bw32) && bw32.blocks <= P->sp.grid_mx) {
                P->box32 = true;
                P->bw32 = bw32;
                P->sp.grid_mx_amul = bw32.blocks;
            }
        }
    }
    P->sp.n_red = m->two_colour ? m->n_red : m->N;
    if (P->rb) {
        // the pair kernels (product, update with the forward sweep, backward
        // sweep): one thread per red-black pair; the |r| and w.r partials of
        // an iteration then number the pair workgroups
        P->sp.grid_amul = cell_blocks(m->n_red);
        P->sp.grid_upd = P->sp.grid_amul;
        // the product, the sweeps, the DIC diagonal and the assembly with two
        // pairs per lane where x-lines hold a multiple of four cells, under the
        // row walk's rule (their partials number their workgroups)
        const RBForm rf = rb_form(m);
        if (rb2_form(rf) && opts.amul_walk != LF_WALK_OFF) {
            const int32_t wb = rb2_blocks(rf.nr);
            if (opts.amul_walk == LF_WALK_ON || wb >= kWalkMinBlocks) {
                P->rb2 = true;
                P->sp.grid_amul = wb;
                P->sp.grid_upd = wb;
            }
        }
    }
    P->fold = opts.precision == LF_PREC_FP64 && opts.precond == LF_PC_DIAGONAL && !P->rb &&
              P->sp.grid_amul <= kFoldPartials && P->sp.grid_upd <= kFoldPartials;
    // larger diagonal FP64 solves on the block walk iterate on the Jacobi-scaled
    // matrix (its coefficients carved by carve_problem for every FP64 diagonal
    // problem of a three-band layout)
    P->scaled = P->box && !P->fold && opts.precision == LF_PREC_FP64 && opts.precond == LF_PC_DIAGONAL;
    P->sp.max_outer = opts.max_outer > 0 ? opts.max_outer : 50;
    P->sp.inner_tol = opts.inner_tol > 0.0 ? opts.inner_tol : 1e-5;
    P->sp.inner_restart = opts.inner_restart ? 1 : 0;
    P->bcs.assign(bcs, bcs + m->P);
    P->ws_bytes = dry.bytes();
    Carver cv(ws);
    carve_problem(cv, m, opts, P);
    auto fail = [&](lf_status st) { lf_problem_destroy(P); return st; };
    std::vector<int32_t> pt(std::max<int32_t>(m->P, 1), 0);
    std::vector<double> pv(std::max<int32_t>(m->P, 1), 0.0);
    for (int32_t p = 0; p < m->P; ++p) { pt[p] = bcs[p].type; pv[p] = bcs[p].value; }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&P->h_state), sizeof(PcgState), hipHostMallocDefault);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventCreate(&P->ev[i]);
    if (e == hipSuccess) e = hipMemcpyAsync(P->patch_type, pt.data(), sizeof(int32_t) * pt.size(), hipMemcpyHostToDevice, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P->patch_value, pv.data(), sizeof(double) * pv.size(), hipMemcpyHostToDevice, P->stream);
    if (e == hipSuccess) e = hipMemsetAsync(P->T, 0, sizeof(double) * m->N, P->stream);
    if (e == hipSuccess) e = hipMemsetAsync(P->state, 0, sizeof(PcgState), P->stream);
    if (e == hipSuccess) e = hipMemsetAsync(P->part, 0, sizeof(double) * kNumPart * P->sp.grid, P->stream);
    // padding entries of the row layout keep coefficient 0 for good; band
    // slots without a face are written as 0 by every assembly
    const size_t slots = coef_slots(m, P->banded, P->rb);
    if (e == hipSuccess) e = hipMemsetAsync(P->coef, 0, sizeof(double) * slots, P->stream);
    if (e == hipSuccess && P->coef32) e = hipMemsetAsync(P->coef32, 0, sizeof(float) * slots, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) { set_error("problem setup failed: %s", hipGetErrorString(e)); return fail(LF_EDEVICE); }
    *out = P;
    return LF_OK;
}

lf_status lf_problem_destroy(lf_problem *P) {
    if (!P) return LF_OK;
    if (P->group) { set_error("the problem is a member of a group until its run finishes"); return LF_ESTATE; }
    if (P->async) {
        if (P->async->active) (void)hipStreamSynchronize(P->stream);   // a run still in flight
        delete P->async;
    }
    for (auto &g : P->g_iter) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : P->g_inner) if (g) (void)hipGraphExecDestroy(g);
    if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
    for (auto &e : P->ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : P->ev_pool) if (e) (void)hipEventDestroy(e);
    if (P->h_state) (void)hipHostFree(P->h_state);
    delete P;
    return LF_OK;
}

lf_status lf_problem_reset(lf_problem *P, const lf_patch_bc *bcs, double DT, double dt) {
    clear_error();
    if (!P) { set_error("problem is NULL"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    const lf_mesh *m = P->mesh;
    LF_TRY(check_physics(m, bcs, DT, dt));
    // DT and dt are kernel arguments; the patch conditions live on the device
    // and are only rewritten (and waited for) when they change
    bool same = static_cast<int32_t>(P->bcs.size()) == m->P;
    for (int32_t p = 0; same && p < m->P; ++p)
        same = P->bcs[p].type == bcs[p].type && std::memcmp(&P->bcs[p].value, &bcs[p].value, sizeof(double)) == 0;
    if (!same) {
        std::vector<int32_t> pt(std::max<int32_t>(m->P, 1), 0);
        std::vector<double> pv(std::max<int32_t>(m->P, 1), 0.0);
        for (int32_t p = 0; p < m->P; ++p) { pt[p] = bcs[p].type; pv[p] = bcs[p].value; }
        LF_HIP(hipMemcpyAsync(P->patch_type, pt.data(), sizeof(int32_t) * pt.size(), hipMemcpyHostToDevice,
                              P->stream));
        LF_HIP(hipMemcpyAsync(P->patch_value, pv.data(), sizeof(double) * pv.size(), hipMemcpyHostToDevice,
                              P->stream));
        LF_HIP(hipStreamSynchronize(P->stream));
    }
    P->bcs.assign(bcs, bcs + m->P);
    P->DT = DT;
    P->dt = dt;
    P->assembled = false;
    P->scaled32 = false;
    P->sumx_valid = false;
    return LF_OK;
}

lf_status lf_problem_layout(const lf_problem *P, int32_t *layout) {
    clear_error();
    if (!P || !layout) { set_error("NULL argument"); return LF_EINVAL; }
    *layout = (P->banded || P->rb) ? LF_LAYOUT_BANDS : LF_LAYOUT_ROWS;
    return LF_OK;
}

lf_status lf_problem_amul_walk(const lf_problem *P, int32_t *walk) {
    clear_error();
    if (!P || !walk) { set_error("NULL argument"); return LF_EINVAL; }
    *walk = P->scaled ? 4 : (P->box ? 2 : (P->walk ? 1 : (P->rb2 ? 3 : 0)));
    return LF_OK;
}

// Cell fields cross the boundary in the mesh's cell order; the solver keeps
// them in its own (lf_mesh::iperm).  y[r] = x[iperm[r]] and y[iperm[r]] = x[r].
__global__ void k_to_solver_order(int32_t n, const int32_t *__restrict__ iperm, const double *__restrict__ x,
                                  double *__restrict__ y) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) y[r] = x[iperm[r]];
}

__global__ void k_to_mesh_order(int32_t n, const int32_t *__restrict__ iperm, const double *__restrict__ x,
                                double *__restrict__ y) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) y[iperm[r]] = x[r];
}

// dst (solver order) from src (mesh order, device), or a copy without a cell order
static lf_status to_solver_order(lf_problem *P, const double *src, double *dst) {
    const lf_mesh *m = P->mesh;
    if (m->iperm)
        hipLaunchKernelGGL(k_to_solver_order, dim3((m->N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream, m->N,
                           m->iperm, src, dst);
    else
        LF_HIP(hipMemcpyAsync(dst, src, sizeof(double) * m->N, hipMemcpyDeviceToDevice, P->stream));
    LF_HIP(hipGetLastError());
    return LF_OK;
}

static lf_status to_mesh_order(lf_problem *P, const double *src, double *dst) {
    const lf_mesh *m = P->mesh;
    if (m->iperm)
        hipLaunchKernelGGL(k_to_mesh_order, dim3((m->N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream, m->N,
                           m->iperm, src, dst);
    else
        LF_HIP(hipMemcpyAsync(dst, src, sizeof(double) * m->N, hipMemcpyDeviceToDevice, P->stream));
    LF_HIP(hipGetLastError());
    return LF_OK;
}

// a solver-order field to host memory in mesh order (through the scratch p2)
static lf_status download_mesh_order(lf_problem *P, const double *src, double *host) {
    const size_t bytes = sizeof(double) * P->mesh->N;
    if (P->mesh->iperm) {
        LF_TRY(to_mesh_order(P, src, P->p2));
        LF_HIP(hipMemcpyAsync(host, P->p2, bytes, hipMemcpyDeviceToHost, P->stream));
    } else {
        LF_HIP(hipMemcpyAsync(host, src, bytes, hipMemcpyDeviceToHost, P->stream));
    }
    return LF_OK;
}

lf_status lf_set_T(lf_problem *P, const double *T, int32_t on_device) {
    clear_error();
    if (!P || !T) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    P->sumx_valid = false;
    const int32_t N = P->mesh->N;
    if (!on_device) {
        for (int32_t c = 0; c < N; ++c)
            if (!std::isfinite(T[c])) { set_error("T[%d] is not finite", c); return LF_EINVAL; }
        if (P->mesh->iperm) {
            LF_HIP(hipMemcpyAsync(P->p2, T, sizeof(double) * N, hipMemcpyHostToDevice, P->stream));
            LF_TRY(to_solver_order(P, P->p2, P->T));
        } else {
            LF_HIP(hipMemcpyAsync(P->T, T, sizeof(double) * N, hipMemcpyHostToDevice, P->stream));
        }
        LF_HIP(hipStreamSynchronize(P->stream));
        return LF_OK;
    }
    bool ok = false;
    LF_TRY(check_finite_device(P, T, &ok));
    if (!ok) { set_error("T holds a non-finite value"); return LF_EINVAL; }
    return to_solver_order(P, T, P->T);
}

lf_status lf_get_T(lf_problem *P, double *T, int32_t on_device) {
    clear_error();
    if (!P || !T) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (on_device) return to_mesh_order(P, P->T, T);
    LF_TRY(download_mesh_order(P, P->T, T));
    LF_HIP(hipStreamSynchronize(P->stream));
    return LF_OK;
}

// field values on the boundary faces: the fixed value on fixedValue patches,
// the face cell's value on zeroGradient patches
__global__ void k_boundary_values(int32_t B, const int32_t *__restrict__ bface_cell,
                                  const int32_t *__restrict__ bface_patch, const int32_t *__restrict__ patch_type,
                                  const double *__restrict__ patch_value, const double *__restrict__ T,
                                  double *__restrict__ Tb) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int32_t pt = bface_patch[b];
    Tb[b] = patch_type[pt] == LF_BC_FIXED_VALUE ? patch_value[pt] : T[bface_cell[b]];
}

lf_status lf_get_boundary_T(lf_problem *P, double *Tb, int32_t on_device) {
    clear_error();
    if (!P || (!Tb && P->mesh->B > 0)) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    const lf_mesh *m = P->mesh;
    if (m->B == 0) return LF_OK;
    double *dst = on_device ? Tb : P->Tb;
    hipLaunchKernelGGL(k_boundary_values, dim3(static_cast<unsigned>((m->B + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       P->stream, m->B, m->rbface_cell, m->bface_patch, P->patch_type, P->patch_value, P->T, dst);
    LF_HIP(hipGetLastError());
    if (!on_device) {
        LF_HIP(hipMemcpyAsync(Tb, P->Tb, sizeof(double) * m->B, hipMemcpyDeviceToHost, P->stream));
        LF_HIP(hipStreamSynchronize(P->stream));
    }
    return LF_OK;
}

lf_status lf_problem_grad(lf_problem *P, double *grad, double *bgrad) {
    clear_error();
    if (!P || !grad) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    return launch_problem_grad(P, grad, bgrad);
}

lf_status lf_assemble(lf_problem *P) {
    clear_error();
    if (!P) { set_error("NULL problem"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    LF_TRY(launch_assemble(P, true, P->stream));
    P->assembled = true;
    return LF_OK;
}

lf_status lf_get_matrix(lf_problem *P, double *diag, double *upper, double *source, double *diag_b,
                        double *source_b, double *int_coeff, double *bou_coeff) {
    clear_error();
    if (!P) { set_error("NULL problem"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (!P->assembled) { set_error("call lf_assemble first"); return LF_ESTATE; }
    const lf_mesh *m = P->mesh;
    hipStream_t s = P->stream;
    const size_t N = m->N, F = m->F, B = m->B;
    (void)N;
    if (diag) LF_TRY(download_mesh_order(P, P->diag, diag));
    if (source) LF_TRY(download_mesh_order(P, P->source, source));
    if (diag_b) LF_TRY(download_mesh_order(P, P->diagB, diag_b));
    if (source_b) LF_TRY(download_mesh_order(P, P->srcB, source_b));
    if (upper && F) LF_HIP(hipMemcpyAsync(upper, P->upper, 8 * F, hipMemcpyDeviceToHost, s));
    if (int_coeff && B) LF_HIP(hipMemcpyAsync(int_coeff, P->int_coeff, 8 * B, hipMemcpyDeviceToHost, s));
    if (bou_coeff && B) LF_HIP(hipMemcpyAsync(bou_coeff, P->bou_coeff, 8 * B, hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    return LF_OK;
}

lf_status lf_amul(lf_problem *P, const double *x, double *y) {
    clear_error();
    if (!P || !x || !y) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (!P->assembled) { set_error("call lf_assemble first"); return LF_ESTATE; }
    if (!P->mesh->iperm) return launch_amul_hook(P, x, y);
    LF_TRY(to_solver_order(P, x, P->p2));
    LF_TRY(launch_amul_hook(P, P->p2, P->q));
    return to_mesh_order(P, P->q, y);
}

lf_status lf_amul_inner(lf_problem *P, const float *x, float *y) {
    clear_error();
    if (!P || !x || !y) { set_error("NULL argument"); return LF_EINVAL; }
    if (P->opts.precision != LF_PREC_MIXED) { set_error("the mixed-precision form's inner product only"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (!P->scaled32) { set_error("no step has formed the FP32 coefficients yet"); return LF_ESTATE; }
    return launch_amul_inner_hook(P, x, y);
}

lf_status lf_precondition(lf_problem *P, const double *r, double *w) {
    clear_error();
    if (!P || !r || !w) { set_error("NULL argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (!P->assembled) { set_error("call lf_assemble first"); return LF_ESTATE; }
    if (P->opts.precision != LF_PREC_FP64) { set_error("the FP64 solver's preconditioner only"); return LF_EINVAL; }
    LF_TRY(to_solver_order(P, r, P->r));
    LF_TRY(launch_precondition_hook(P));
    return to_mesh_order(P, P->w, w);
}

lf_status lf_profile_enable(lf_problem *P, int32_t on) {
    clear_error();
    if (!P) { set_error("NULL problem"); return LF_EINVAL; }
    P->prof_on = on != 0;
    for (int k = 0; k < LF_NUM_KERNEL_CLASSES; ++k) { P->prof_ms[k] = 0.0; P->prof_n[k] = 0; }
    P->prof_pending.clear();
    P->ev_used = 0;
    return LF_OK;
}

lf_status lf_profile_read(lf_problem *P, int32_t n, double *total_ms, int64_t *launches) {
    clear_error();
    if (!P || n < 0) { set_error("bad argument"); return LF_EINVAL; }
    for (int32_t k = 0; k < n; ++k) {
        if (total_ms) total_ms[k] = k < LF_NUM_KERNEL_CLASSES ? P->prof_ms[k] : 0.0;
        if (launches) launches[k] = k < LF_NUM_KERNEL_CLASSES ? P->prof_n[k] : 0;
    }
    return LF_OK;
}

// One problem's time steps as a sequence of enqueue / advance phases (see
// SolveCtx); lf_step drives one, lf_step_many several at once.


static int32_t corrector_passes(const lf_problem *P) { return P->nonorth ? P->opts.n_nonorth_corr : 0; }

// one assembly + solve: the step's only pass, or one pass of its
// non-orthogonal corrector loop
static lf_status begin_pass(StepDriver &d) {
    lf_problem *P = d.P;
    hipStream_t s = P->stream;
    std::memset(&d.cur, 0, sizeof(d.cur));
    prof_lead(P, s);
    LF_HIP(hipEventRecord(P->ev[0], s));
    LF_TRY(launch_assemble_setup(P, s));
    LF_HIP(hipEventRecord(P->ev[1], s));
    P->assembled = true;
    return P->opts.precision == LF_PREC_MIXED ? mixed_start(P, d.c) : fp64_start(P, d.c);
}

static lf_status begin_step(StepDriver &d) {
    lf_problem *P = d.P;
    d.pass = 0;
    std::memset(&d.acc, 0, sizeof(d.acc));
    // the corrector passes take their ddt source from T at the start of the step
    if (corrector_passes(P) > 0)
        LF_HIP(hipMemcpyAsync(P->T_old, P->T, sizeof(double) * P->mesh->N, hipMemcpyDeviceToDevice, P->stream));
    return begin_pass(d);
}

// called once P->ev[2] has completed
static lf_status advance(StepDriver &d) {
    lf_problem *P = d.P;
    bool done = false;
    LF_TRY(P->opts.precision == LF_PREC_MIXED ? mixed_advance(P, d.c, &done, &d.cur)
                                              : fp64_advance(P, d.c, &done, &d.cur));
    if (!done) return LF_OK;
    float a_ms = 0.f, s_ms = 0.f;
    LF_HIP(hipEventElapsedTime(&a_ms, P->ev[0], P->ev[1]));
    LF_HIP(hipEventElapsedTime(&s_ms, P->ev[1], P->ev[2]));
    d.cur.assemble_ms = a_ms;
    d.cur.solve_ms = s_ms;
    P->last_iters = d.cur.n_iter;
    if (!d.cur.nonfinite && d.pass < corrector_passes(P)) {
        // the next pass of the corrector loop from the T just solved for
        if (d.pass == 0) d.acc.initial_residual = d.cur.initial_residual;
        d.acc.n_iter += d.cur.n_iter;
        d.acc.n_outer += d.cur.n_outer;
        d.acc.assemble_ms += d.cur.assemble_ms;
        d.acc.solve_ms += d.cur.solve_ms;
        ++d.pass;
        return begin_pass(d);
    }
    if (d.pass > 0) {
        // the step's stats: the first pass's initial residual, the last pass's
        // final residual and flags, iterations and times summed over the passes
        d.cur.initial_residual = d.acc.initial_residual;
        d.cur.n_iter += d.acc.n_iter;
        d.cur.n_outer += d.acc.n_outer;
        d.cur.assemble_ms += d.acc.assemble_ms;
        d.cur.solve_ms += d.acc.solve_ms;
    }
    if (d.stats) d.stats[d.step] = d.cur;
    // T of this step into its snapshot, on the stream before the next step's work
    if (d.snap) LF_TRY(to_mesh_order(P, P->T, d.snap + static_cast<int64_t>(d.step) * P->mesh->N));
    ++d.step;
    if (d.cur.nonfinite) {
        d.nonfinite = true;
        d.active = false;
        return LF_OK;
    }
    if (d.step < d.n_steps) return begin_step(d);
    d.active = false;
    return LF_OK;
}

lf_status lf_step(lf_problem *P, int32_t n_steps, lf_solve_stats *stats) {
    clear_error();
    if (!P || n_steps < 0) { set_error("bad argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (n_steps == 0) return LF_OK;
    StepDriver d;
    d.P = P;
    d.stats = stats;
    d.n_steps = n_steps;
    d.active = true;
    LF_TRY(begin_step(d));
    while (d.active) {
        LF_HIP(hipEventSynchronize(P->ev[2]));
        LF_TRY(advance(d));
    }
    if (d.nonfinite) { set_error("non-finite residual in step %d", d.step - 1); return LF_ENONFINITE; }
    return LF_OK;
}

lf_status lf_step_many(lf_problem *const *problems, int32_t n, int32_t n_steps, lf_solve_stats *stats) {
    clear_error();
    if (!problems || n < 1 || n_steps < 0) { set_error("bad argument"); return LF_EINVAL; }
    for (int32_t i = 0; i < n; ++i) {
        if (!problems[i]) { set_error("problem %d is NULL", i); return LF_EINVAL; }
        if (async_running(problems[i])) { set_error("problem %d: an lf_step_begin run is in flight", i); return LF_ESTATE; }
        for (int32_t j = 0; j < i; ++j)
            if (problems[j] == problems[i]) { set_error("problem %d given twice", i); return LF_EINVAL; }
    }
    if (n_steps == 0) return LF_OK;
    std::vector<StepDriver> ds(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) {
        ds[i].P = problems[i];
        ds[i].stats = stats ? stats + static_cast<int64_t>(i) * n_steps : nullptr;
        ds[i].n_steps = n_steps;
        ds[i].active = true;
        LF_TRY(begin_step(ds[i]));
    }
    // advance whichever problem's last enqueued block has finished; every
    // active problem always has work queued on its stream
    for (int32_t active = n; active > 0;) {
        bool progressed = false;
        for (auto &d : ds) {
            if (!d.active) continue;
            const hipError_t q = hipEventQuery(d.P->ev[2]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) { set_error("hipEventQuery failed: %s", hipGetErrorString(q)); return LF_EDEVICE; }
            LF_TRY(advance(d));
            progressed = true;
            if (!d.active) --active;
        }
        if (!progressed) std::this_thread::yield();
    }
    for (int32_t i = 0; i < n; ++i)
        if (ds[i].nonfinite) {
            set_error("problem %d: non-finite residual in step %d", i, ds[i].step - 1);
            return LF_ENONFINITE;
        }
    return LF_OK;
}

lf_status lf_step_begin(lf_problem *P, int32_t n_steps, double *snapshots) {
    clear_error();
    if (!P || n_steps < 1) { set_error("bad argument"); return LF_EINVAL; }
    if (async_running(P)) { set_error("a run is in flight (lf_step_begin or a group)"); return LF_ESTATE; }
    if (!P->async) {
        P->async = new (std::nothrow) StepDriver();
        if (!P->async) { set_error("host allocation failed"); return LF_ENOMEM; }
    }
    StepDriver &d = *P->async;
    d.own_stats.assign(static_cast<size_t>(n_steps), lf_solve_stats{});
    d.P = P;
    d.stats = d.own_stats.data();
    d.snap = snapshots;
    d.n_steps = n_steps;
    d.step = 0;
    d.nonfinite = false;
    d.active = true;
    const lf_status st = begin_step(d);
    if (st != LF_OK) d.active = false;
    return st;
}

lf_status lf_step_poll(lf_problem *P, int32_t *steps_done, int32_t *finished, lf_solve_stats *stats) {
    clear_error();
    if (!P || !steps_done || !finished) { set_error("NULL argument"); return LF_EINVAL; }
    if (!P->async) { set_error("no lf_step_begin run"); return LF_ESTATE; }
    StepDriver &d = *P->async;
    while (d.active) {
        const hipError_t q = hipEventQuery(P->ev[2]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            d.active = false;
            set_error("hipEventQuery failed: %s", hipGetErrorString(q));
            return LF_EDEVICE;
        }
        const lf_status st = advance(d);
        if (st != LF_OK) { d.active = false; return st; }
    }
    *steps_done = d.step;
    *finished = d.active ? 0 : 1;
    if (stats && d.step > 0) std::memcpy(stats, d.own_stats.data(), sizeof(lf_solve_stats) * d.step);
    if (!d.active && d.nonfinite) {
        set_error("non-finite residual in step %d", d.step - 1);
        return LF_ENONFINITE;
    }
    return LF_OK;
}

}  // extern "C"
