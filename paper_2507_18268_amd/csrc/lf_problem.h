// Problem handle: one mesh + boundary conditions + DT + dt + solver options.
#pragma once

#include "lf_internal.h"

namespace lf {

// Slots of the per-workgroup partial sums (deterministic two-stage reductions).
enum PartialSlot : int {
    kPartSumX = 0,   // sum of x0 (mean for the normalisation factor)
    kPartSumR = 1,   // sum |r|
    kPartNf = 2,     // sum |A x0 - pA| + |b - pA|
    kPartWr = 3,     // sum w.r
    kPartPq = 4,     // sum p.Ap
    kNumPart = 5
};

// Solver state on the device.  Written only by workgroup 0 of a kernel; every
// workgroup recomputes the same scalars from the same partials, so no
// workgroup ever waits for another inside a kernel.
struct PcgState {
    double nf;            // normalisation factor
    double res0;          // initial normalised residual
    double res;           // current normalised residual
    double wArA_cur;      // w.r of the current iteration (read by the update kernel)
    double wArA_slot[2];  // w.r by iteration parity (read by the next direction update)
    double alpha;         // last step length (diagnostics)
    int32_t n_iter;
    int32_t done;
    int32_t converged;
    int32_t singular;
    int32_t nonfinite;
    int32_t flag;         // scratch flag (input checks)
};

struct SolverParams {
    double tol, rel_tol;
    int32_t max_iter, min_iter;
    int32_t n;            // cells
    int32_t chunk;        // cells per workgroup
    int32_t grid;         // workgroups
    int32_t n_red;        // DIC: first black cell
};

}  // namespace lf

struct lf_problem {
    const lf_mesh *mesh = nullptr;
    lf_solver_opts opts{};
    double DT = 0, dt = 0;
    hipStream_t stream = nullptr;
    lf::CellGrid grid{};
    lf::SolverParams sp{};
    std::vector<lf_patch_bc> bcs;
    // device arrays (caller workspace)
    int32_t *patch_type = nullptr;
    double *patch_value = nullptr;
    double *T = nullptr;                       // [N] the field; PCG solves in place
    double *r = nullptr, *p = nullptr, *q = nullptr, *w = nullptr, *rD = nullptr, *sumA = nullptr;
    double *diag = nullptr, *source = nullptr, *diagB = nullptr, *srcB = nullptr;
    double *upper = nullptr, *coef = nullptr;  // [F] face order, [2F] row order
    double *int_coeff = nullptr, *bou_coeff = nullptr;
    double *part = nullptr;                    // [kNumPart][kMaxGrid]
    lf::PcgState *state = nullptr;
    // mixed precision (FP32 inner solve)
    float *coef32 = nullptr, *diag32 = nullptr, *rD32 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    // host side
    lf::PcgState *h_state = nullptr;           // pinned
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t g_iter[8] = {};             // (KA, KU, KP) x 2^i
    hipGraphExec_t g_prologue = nullptr;
    int32_t last_iters = 0;
    bool assembled = false;
    size_t ws_bytes = 0;
};
