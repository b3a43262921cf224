// Precision form: mixed-precision iterative refinement.
//
// The matrix is assembled in FP64 (with an FP32 copy of its coefficients).
// Outer loop in FP64: r = b - A T (true residual, FP64 coefficients and T),
// res = sum|r| / normFactor with the normalisation factor of x0 = T_old, stop
// when res < tol.  Each pass solves A d = r approximately with a PCG whose
// vectors, coefficients and products are FP32, while its dot products, alpha
// and beta are FP64; then T += d in FP64.  The inner solve of a pass stops
// when its L1 residual has fallen by inner_tol, or below half the outer
// target, whichever is larger.
//
// The refinement runs until res < kTighten * tol (convergence is still
// reported against tol).  Every FP64 PCG that stops just below tol leaves an
// error of its own in T (up to ~6e-9 relative per step on these meshes); by
// stopping an order of magnitude lower the precision form stays within 1e-8
// of such a solve of the same system.
constexpr double kTighten = 0.1;
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lf_solver.h"

namespace lf {

void carve_mixed(Carver &cv, const lf_mesh *m, bool banded, lf_problem *P) {
    const size_t N = m->N;
    auto *coef32 = cv.take<float>(coef_slots(m, banded));
    float *v32[6];
    for (auto &v : v32) v = cv.take<float>(N);
    if (P) {
        P->coef32 = coef32; P->diag32 = v32[0]; P->rD32 = v32[1]; P->r32 = v32[2];
        P->p32 = v32[3]; P->q32 = v32[4]; P->d32 = v32[5];
    }
}

__device__ __forceinline__ bool inner_off(const PcgState *st) { return st->done || st->inner_done; }

// p = w (first inner iteration) or w + beta p, w = rD r, all FP32
__global__ void __launch_bounds__(kCellBlock)
k_mx_direction(SolverParams sp, const float *__restrict__ rD32, const float *__restrict__ r32,
               float *__restrict__ p32, const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    const bool first = st->inner_iter == 0;
    const float beta = static_cast<float>(st->beta);
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row<kMxRows>(j);
        if (c >= sp.n) continue;
        const float wc = rD32[c] * r32[c];
        p32[c] = first ? wc : wc + beta * p32[c];
    }
}

// q = A p in FP32; FP64 partial sums of p.q
template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_amul_dot(SolverParams sp, Lay L, const float *__restrict__ diag32, const float *__restrict__ coef32,
              const float *__restrict__ p32, float *__restrict__ q32, double *__restrict__ part,
              const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    double acc[1] = {0.0};
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row<kMxRows>(j);
        if (c >= sp.n) continue;
        const float pc = p32[c];
        const float qc = layout_dot(L, c, coef32, p32, diag32[c] * pc);
        q32[c] = qc;
        acc[0] += static_cast<double>(qc) * static_cast<double>(pc);
    }
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid_mx, slots, acc);
}

// d += alpha p; r -= alpha q (FP32); FP64 partials of |r| and w.r
__global__ void __launch_bounds__(kCellBlock)
k_mx_update(SolverParams sp, const float *__restrict__ p32, const float *__restrict__ q32,
            const float *__restrict__ rD32, float *__restrict__ r32, float *__restrict__ d32,
            double *__restrict__ part, const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    const float alpha = static_cast<float>(st->alpha);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row<kMxRows>(j);
        if (c >= sp.n) continue;
        d32[c] += alpha * p32[c];
        const float rc = r32[c] - alpha * q32[c];
        r32[c] = rc;
        const float wc = rD32[c] * rc;
        acc[0] += fabs(static_cast<double>(rc));
        acc[1] += static_cast<double>(wc) * static_cast<double>(rc);
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials<2>(part, sp.grid_mx, slots, acc);
}

// T += d (FP64)
__global__ void __launch_bounds__(kCellBlock)
k_mx_correct(SolverParams sp, double *__restrict__ T, const float *__restrict__ d32, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) T[c] += static_cast<double>(d32[c]);
}

// true residual r = b - A T in FP64 and its partial sums of |r|; also the
// start of the next pass, which runs if the outer check does not stop the
// solve: r32 = r rounded to FP32, d = 0, partial sums of |r32| and w32.r32
template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_residual(SolverParams sp, Lay L, const double *__restrict__ diagB, const double *__restrict__ coef,
              const double *__restrict__ srcB, const double *__restrict__ T, double *__restrict__ r,
              const float *__restrict__ rD32, float *__restrict__ r32, float *__restrict__ d32,
              double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[3] = {0.0, 0.0, 0.0};
    if (c < sp.n) {
        const double ax = layout_dot(L, c, coef, T, diagB[c] * T[c]);
        const double rc = srcB[c] - ax;
        r[c] = rc;
        acc[0] = fabs(rc);
        const float r32c = static_cast<float>(rc);
        r32[c] = r32c;
        d32[c] = 0.0f;
        const float w32 = rD32[c] * r32c;
        acc[1] = fabs(static_cast<double>(r32c));
        acc[2] = static_cast<double>(w32) * static_cast<double>(r32c);
    }
    const int slots[3] = {kPartSumR, kPartSumR32, kPartWr32};
    write_partials<3>(part, sp.grid, slots, acc);
}

// one-workgroup decisions of the refinement
enum MxFin : int { kMxInnerStart = 0, kMxAlpha = 1, kMxBeta = 2, kMxOuter = 3 };

template <int Mode>
__global__ void __launch_bounds__(kFinBlock) k_mx_finalize(SolverParams sp, const double *__restrict__ part,
                                                          PcgState *__restrict__ st) {
    // partials per slot: the FP32 inner kernels use their own grid
    const int32_t G = (Mode == kMxAlpha || Mode == kMxBeta) ? sp.grid_mx : sp.grid;
    if (Mode == kMxInnerStart) {
        if (st->done) return;
        double v[2];
        const int slots[2] = {kPartSumR32, kPartWr32};
        reduce_partials<2>(part, G, slots, v);
        if (threadIdx.x == 0) {
            const double target = fmax(sp.inner_tol * v[0], 0.5 * kTighten * sp.tol * st->nf);
            st->inner_target = target;
            st->inner_iter = 0;
            st->wArA = v[1];
            st->inner_done = (v[0] <= target || !(v[1] > 0.0)) ? 1 : 0;
            if (!isfinite(v[0]) || !isfinite(v[1])) {
                st->nonfinite = 1;
                st->done = 1;
            }
        }
    } else if (Mode == kMxAlpha) {
        if (inner_off(st)) return;
        double v[1];
        const int slots[1] = {kPartPq};
        reduce_partials<1>(part, G, slots, v);
        if (threadIdx.x == 0) {
            const double pq = v[0];
            if (!isfinite(pq)) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (!(fabs(pq) > 0.0)) {
                st->inner_done = 1;          // nothing left that FP32 can resolve
            } else {
                st->alpha = st->wArA / pq;
            }
        }
    } else if (Mode == kMxBeta) {
        if (inner_off(st)) return;
        double v[2];
        const int slots[2] = {kPartSumR, kPartWr};
        reduce_partials<2>(part, G, slots, v);
        if (threadIdx.x == 0) {
            st->inner_iter += 1;
            st->n_iter += 1;
            if (!isfinite(v[0]) || !isfinite(v[1])) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (v[0] <= st->inner_target || st->n_iter >= sp.max_iter || !(v[1] > 0.0)) {
                st->inner_done = 1;
            } else {
                st->beta = v[1] / st->wArA;
                st->wArA = v[1];
            }
        }
    } else {
        if (st->done) return;
        double v[1];
        const int slots[1] = {kPartSumR};
        reduce_partials<1>(part, G, slots, v);
        if (threadIdx.x == 0) {
            const double res = v[0] / st->nf;
            st->res = res;
            st->n_outer += 1;
            const bool conv = check_conv(res, st->res0, sp.tol, sp.rel_tol);
            const bool tight = check_conv(res, st->res0, kTighten * sp.tol, kTighten * sp.rel_tol);
            st->converged = conv ? 1 : 0;
            if (!isfinite(res)) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (tight || st->n_outer >= sp.max_outer || st->n_iter >= sp.max_iter) {
                st->done = 1;
            }
        }
    }
}

template <int Mode>
static void launch_mx_fin(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_FINALIZE, s, k_mx_finalize<Mode>, dim3(1), dim3(kFinBlock), 0, s, P->sp, P->part, P->state);
}

static void launch_inner_iteration(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_INNER_DIRECTION, s, k_mx_direction, mx_grid(P), dim3(kCellBlock), 0, s, P->sp, P->rD32,
              P->r32, P->p32, P->state);
    with_layout(P, [&](auto lay) {
        LF_LAUNCH(P, LF_K_INNER_AMUL_DOT, s, k_mx_amul_dot<decltype(lay)>, mx_grid(P), dim3(kCellBlock), 0, s,
                  P->sp, lay, P->diag32, P->coef32, P->p32, P->q32, P->part, P->state);
    });
    launch_mx_fin<kMxAlpha>(P, s);
    LF_LAUNCH(P, LF_K_INNER_UPDATE, s, k_mx_update, mx_grid(P), dim3(kCellBlock), 0, s, P->sp, P->p32, P->q32,
              P->rD32, P->r32, P->d32, P->part, P->state);
    launch_mx_fin<kMxBeta>(P, s);
}

// start of a refinement pass (r32, d = 0 and their partial sums were written
// by the kernel that formed the FP64 residual: the assembly or k_mx_residual)
static void launch_pass_start(lf_problem *P, hipStream_t s) { launch_mx_fin<kMxInnerStart>(P, s); }

// end of a pass: correction, true residual, outer decision
static void launch_pass_end(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_MIXED_CORRECT, s, k_mx_correct, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->T, P->d32,
              P->state);
    with_layout(P, [&](auto lay) {
        LF_LAUNCH(P, LF_K_MIXED_RESIDUAL, s, k_mx_residual<decltype(lay)>, cell_grid(P), dim3(kCellBlock), 0, s,
                  P->sp, lay, P->diagB, P->coef, P->srcB, P->T, P->r, P->rD32, P->r32, P->d32, P->part,
                  P->state);
    });
    launch_mx_fin<kMxOuter>(P, s);
}

static lf_status get_inner_graph(lf_problem *P, int lg) {
    if (P->g_inner[lg]) return LF_OK;
    if (!P->capture_stream) LF_HIP(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = P->capture_stream;
    LF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < (1 << lg); ++i) launch_inner_iteration(P, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess) { set_error("graph capture failed: %s", hipGetErrorString(e)); return LF_EDEVICE; }
    e = hipGraphInstantiate(&P->g_inner[lg], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { set_error("graph instantiate failed: %s", hipGetErrorString(e)); return LF_EDEVICE; }
    return LF_OK;
}

static lf_status launch_inner(lf_problem *P, int32_t k) {
    hipStream_t s = P->stream;
    if (!P->opts.use_graph || P->prof_on) {
        for (int32_t i = 0; i < k; ++i) launch_inner_iteration(P, s);
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    for (int lg = kMaxGraphLog; lg >= 0; --lg) {
        while (k >= (1 << lg)) {
            LF_TRY(get_inner_graph(P, lg));
            LF_HIP(hipGraphLaunch(P->g_inner[lg], s));
            k -= 1 << lg;
        }
    }
    return LF_OK;
}

// block of k inner iterations, then the state copy and ev[2]
static lf_status mixed_block(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    prof_lead(P, s);
    LF_TRY(launch_inner(P, c.k));
    c.launched += c.k;
    LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    LF_HIP(hipEventRecord(P->ev[2], s));
    return LF_OK;
}

lf_status mixed_start(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    prof_lead(P, s);
    launch_fin<kFinStart>(P, s);      // normFactor, res0 and the initial decision (shared with FP64)
    launch_pass_start(P, s);
    LF_HIP(hipGetLastError());
    c.fixed_k = P->prof_on ? 1 : P->opts.iters_per_check;
    c.k = c.fixed_k > 0 ? c.fixed_k : std::max<int32_t>(2, P->last_inner > 0 ? P->last_inner : 8);
    c.launched = 0;
    return mixed_block(P, c);
}

lf_status mixed_advance(lf_problem *P, SolveCtx &c, bool *finished, lf_solve_stats *out) {
    hipStream_t s = P->stream;
    prof_flush(P);
    *finished = false;
    const PcgState &h = *P->h_state;
    if (h.done) {
        out->initial_residual = h.res0;
        out->final_residual = h.res;
        out->n_iter = h.n_iter;
        out->converged = h.converged;
        out->singular = 0;
        out->nonfinite = h.nonfinite;
        out->n_outer = h.n_outer;
        *finished = true;
        return LF_OK;
    }
    if (c.launched > 4 * (P->sp.max_iter + 8) + 64 * P->sp.max_outer) {
        set_error("mixed solver never reached done after %d launched inner iterations", c.launched);
        return LF_ESTATE;
    }
    if (!h.inner_done) {
        if (c.fixed_k <= 0) c.k = std::max<int32_t>(2, c.k / 2);
    } else {
        // pass finished: correct, check, start the next pass (no-ops once done)
        if (c.fixed_k <= 0) {
            c.k = std::max<int32_t>(2, h.inner_iter);
            P->last_inner = h.inner_iter;
        }
        prof_lead(P, s);
        launch_pass_end(P, s);
        launch_pass_start(P, s);
        LF_HIP(hipGetLastError());
    }
    return mixed_block(P, c);
}

}  // namespace lf
