// Per-step assembly of TEqn = ddt(T) - laplacian(DT, T) and its PCG solve.
//
// Every kernel is cell-parallel over contiguous cell chunks (one chunk per
// workgroup, XCD-aware), gathers through the row-ordered off-diagonal lists
// (no atomics, so results are deterministic), and reduces through per-workgroup
// partials that the next kernel sums in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "lf_kernels.h"

namespace lf {

// ---------------------------------------------------------------------------
// assembly (Listing 1): upper_f = -(delta_f (DT |S_f|)), diag = V/dt - lapDiag
// with lapDiag the negated sum of the Laplacian face coefficients of the row in
// face order, source = (T_old/dt) V; fixedValue faces add (DT|S_b|) delta_b to
// the diagonal and (DT|S_b|)(delta_b T_b) to the source.
// kFull also stores diag/source without the boundary part (test hook).
// ---------------------------------------------------------------------------
template <bool kFull>
__global__ void __launch_bounds__(kBlock)
k_assemble(SolverParams sp, double rdt, double DT, const int32_t *__restrict__ row_start,
           const int32_t *__restrict__ face_of, const int32_t *__restrict__ owner_start,
           const double *__restrict__ mag_sf, const double *__restrict__ delta,
           const int32_t *__restrict__ bface_start, const int32_t *__restrict__ bface_list,
           const int32_t *__restrict__ bface_patch, const double *__restrict__ bmag_sf,
           const double *__restrict__ bdelta, const int32_t *__restrict__ patch_type,
           const double *__restrict__ patch_value, const double *__restrict__ V,
           const double *__restrict__ T, double *__restrict__ coef, double *__restrict__ upper,
           double *__restrict__ diag, double *__restrict__ source, double *__restrict__ diagB,
           double *__restrict__ srcB, double *__restrict__ int_coeff, double *__restrict__ bou_coeff) {
    const CellRange cr = cell_range(sp.n, sp.chunk, logical_block());
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const int32_t e0 = row_start[c], e1 = row_start[c + 1];
        const int32_t first_up = e1 - (owner_start[c + 1] - owner_start[c]);
        double lap_diag = 0.0;
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t f = face_of[e];
            const double lap_upper = delta[f] * (DT * mag_sf[f]);
            coef[e] = -lap_upper;
            lap_diag -= lap_upper;
            if (e >= first_up) upper[f] = -lap_upper;
        }
        const double v = V[c];
        const double d = rdt * v - lap_diag;
        const double s = (rdt * T[c]) * v;
        double db = d, sb = s;
        for (int32_t i = bface_start[c]; i < bface_start[c + 1]; ++i) {
            const int32_t b = bface_list[i];
            const int32_t pt = bface_patch[b];
            if (patch_type[pt] == LF_BC_FIXED_VALUE) {
                const double g = DT * bmag_sf[b];
                const double ic = g * bdelta[b];
                const double bc = g * (bdelta[b] * patch_value[pt]);
                db += ic;
                sb += bc;
                if (kFull) { int_coeff[b] = ic; bou_coeff[b] = bc; }
            } else if (kFull) {
                int_coeff[b] = 0.0;
                bou_coeff[b] = 0.0;
            }
        }
        if (kFull) { diag[c] = d; source[c] = s; }
        diagB[c] = db;
        srcB[c] = sb;
    }
}

// ---------------------------------------------------------------------------
// LDU product y = A x in the order of a sequential face loop: diag x first,
// then the row's lower faces ascending, then its owned faces ascending.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double row_amul(int32_t c, const double *__restrict__ diagB,
                                           const double *__restrict__ coef,
                                           const int32_t *__restrict__ row_start,
                                           const int32_t *__restrict__ col,
                                           const double *__restrict__ x) {
    double acc = diagB[c] * x[c];
    const int32_t e1 = row_start[c + 1];
    for (int32_t e = row_start[c]; e < e1; ++e) acc += coef[e] * x[col[e]];
    return acc;
}

__global__ void __launch_bounds__(kBlock)
k_amul(SolverParams sp, const double *__restrict__ diagB, const double *__restrict__ coef,
       const int32_t *__restrict__ row_start, const int32_t *__restrict__ col,
       const double *__restrict__ x, double *__restrict__ y) {
    const CellRange cr = cell_range(sp.n, sp.chunk, logical_block());
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock)
        y[c] = row_amul(c, diagB, coef, row_start, col, x);
}

// ---------------------------------------------------------------------------
// PCG setup: wA = A x0, r = b - wA, row sums of A, rD = 1/diag (diagonal
// preconditioner); partial sums of x0 and |r|.  Resets the solver state.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_setup1(SolverParams sp, int32_t diag_pc, const double *__restrict__ diagB, const double *__restrict__ coef,
         const int32_t *__restrict__ row_start, const int32_t *__restrict__ col,
         const double *__restrict__ x, const double *__restrict__ srcB, double *__restrict__ q,
         double *__restrict__ r, double *__restrict__ sumA, double *__restrict__ rD,
         double *__restrict__ part, PcgState *__restrict__ st) {
    const int32_t L = logical_block();
    const CellRange cr = cell_range(sp.n, sp.chunk, L);
    double acc[2] = {0.0, 0.0};
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const double d = diagB[c];
        const double xc = x[c];
        double ax = d * xc, sa = d;
        const int32_t e1 = row_start[c + 1];
        for (int32_t e = row_start[c]; e < e1; ++e) {
            const double a = coef[e];
            ax += a * x[col[e]];
            sa += a;
        }
        const double rc = srcB[c] - ax;
        q[c] = ax;
        r[c] = rc;
        sumA[c] = sa;
        if (diag_pc) rD[c] = 1.0 / d;
        acc[0] += xc;
        acc[1] += fabs(rc);
    }
    const int slots[2] = {kPartSumX, kPartSumR};
    write_partials<2>(part, slots, acc, L);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_iter = 0;
        st->done = 0;
        st->converged = 0;
        st->singular = 0;
        st->nonfinite = 0;
        st->alpha = 0.0;
    }
}

// normalisation factor terms |wA - pA| + |b - pA| with pA = sumA * mean(x0);
// with the diagonal preconditioner also the first w.r.
__global__ void __launch_bounds__(kBlock)
k_setup2(SolverParams sp, int32_t diag_pc, const double *__restrict__ sumA, const double *__restrict__ q,
         const double *__restrict__ srcB, const double *__restrict__ rD, const double *__restrict__ r,
         double *__restrict__ part) {
    const int32_t L = logical_block();
    double sx[1];
    const int sslot[1] = {kPartSumX};
    reduce_partials<1>(part, sslot, sp.grid, sx);
    const double x_avg = sx[0] / static_cast<double>(sp.n);
    const CellRange cr = cell_range(sp.n, sp.chunk, L);
    double acc[2] = {0.0, 0.0};
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const double pa = sumA[c] * x_avg;
        acc[0] += fabs(q[c] - pa) + fabs(srcB[c] - pa);
        if (diag_pc) {
            const double rc = r[c];
            const double wc = rD[c] * rc;
            acc[1] += wc * rc;
        }
    }
    const int slots[2] = {kPartNf, kPartWr};
    write_partials<2>(part, slots, acc, L);
}

// ---------------------------------------------------------------------------
// Direction update (start of a PCG iteration): finish the residual reduction
// of the previous update, make the convergence decision, then
// p = w (first iteration) or p = w + beta p, beta = wArA / wArA_old,
// w = rD r (diagonal) or the stored preconditioned residual (DIC).
// ---------------------------------------------------------------------------
template <bool kDiag>
__global__ void __launch_bounds__(kBlock)
k_direction(SolverParams sp, const double *__restrict__ rD, const double *__restrict__ r,
            const double *__restrict__ w, double *__restrict__ p, const double *__restrict__ part,
            PcgState *__restrict__ st) {
    const StateView sv = load_state(st);
    if (sv.done) return;
    const int32_t k = sv.n_iter;
    const bool first = (k == 0);
    double sums[3];
    const int slots[3] = {kPartSumR, kPartWr, kPartNf};
    reduce_partials<3>(part, slots, sp.grid, sums);
    const double nf = first ? sums[2] + 1e-20 : sv.nf;
    const double res = sums[0] / nf;
    const double res0 = first ? res : sv.res0;
    bool conv;
    bool cont;
    if (first) {
        conv = check_conv(res, res, sp.tol, sp.rel_tol);
        cont = sp.min_iter > 0 || !conv;
    } else {
        conv = (k < sp.max_iter) ? check_conv(res, res0, sp.tol, sp.rel_tol) : (sv.converged != 0);
        cont = (k < sp.max_iter && !conv) || k < sp.min_iter;
    }
    const bool bad = !isfinite(res) || !isfinite(sums[1]);
    const double wr = sums[1];
    if (!cont || bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (first) { st->nf = nf; st->res0 = res; }
            st->res = res;
            st->converged = conv ? 1 : 0;
            st->nonfinite = bad ? 1 : 0;
            st->done = 1;
        }
        return;
    }
    const double beta = first ? 0.0 : wr / sv.wArA_prev;
    const CellRange cr = cell_range(sp.n, sp.chunk, logical_block());
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const double wc = kDiag ? rD[c] * r[c] : w[c];
        p[c] = first ? wc : wc + beta * p[c];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) { st->nf = nf; st->res0 = res; }
        st->res = res;
        st->converged = conv ? 1 : 0;
        st->wArA_cur = wr;
        st->wArA_slot[k & 1] = wr;
    }
}

// q = A p and the partial sums of q.p
__global__ void __launch_bounds__(kBlock)
k_amul_dot(SolverParams sp, const double *__restrict__ diagB, const double *__restrict__ coef,
           const int32_t *__restrict__ row_start, const int32_t *__restrict__ col,
           const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
           const PcgState *__restrict__ st) {
    if (load_state(st).done) return;
    const int32_t L = logical_block();
    const CellRange cr = cell_range(sp.n, sp.chunk, L);
    double acc[1] = {0.0};
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const double qc = row_amul(c, diagB, coef, row_start, col, p);
        q[c] = qc;
        acc[0] += qc * p[c];
    }
    const int slots[1] = {kPartPq};
    write_partials<1>(part, slots, acc, L);
}

// alpha = wArA / p.Ap (singular if |p.Ap|/nf < 1e-300); x += alpha p;
// r -= alpha q; partial sums of |r| and (diagonal) of w.r with w = rD r.
template <bool kDiag>
__global__ void __launch_bounds__(kBlock)
k_update(SolverParams sp, double *__restrict__ x, const double *__restrict__ p, const double *__restrict__ q,
         double *__restrict__ r, const double *__restrict__ rD, double *__restrict__ part,
         PcgState *__restrict__ st) {
    const StateView sv = load_state(st);
    if (sv.done) return;
    double pq[1];
    const int pslot[1] = {kPartPq};
    reduce_partials<1>(part, pslot, sp.grid, pq);
    const double nf = sv.nf;
    const bool bad = !isfinite(pq[0]);
    if (bad || fabs(pq[0]) / nf < 1e-300) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (bad) st->nonfinite = 1; else st->singular = 1;
            st->done = 1;
        }
        return;
    }
    const double alpha = sv.wArA_cur / pq[0];
    const int32_t L = logical_block();
    const CellRange cr = cell_range(sp.n, sp.chunk, L);
    double acc[2] = {0.0, 0.0};
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        x[c] += alpha * p[c];
        const double rc = r[c] - alpha * q[c];
        r[c] = rc;
        acc[0] += fabs(rc);
        if (kDiag) {
            const double wc = rD[c] * rc;
            acc[1] += wc * rc;
        }
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials<2>(part, slots, acc, L);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_iter = sv.n_iter + 1;
        st->alpha = alpha;
    }
}

// ---------------------------------------------------------------------------
// DIC on a two-colour numbering (cells [0, n_red) red, [n_red, N) black; every
// face has a red owner and a black neighbour).  The sequential DIC recurrences
// then become cell-parallel gathers in the same order:
//   rD_red = diag, rD_black = diag - sum over its lower faces (ascending) of
//   upper^2 / rD_owner;  rD = 1/rD.
//   forward:  w_b = rD_b r_b - sum over lower faces (ascending) (rD_b upper) w_o
//             with w_o = rD_o r_o for the red owners
//   backward: w_r = rD_r r_r - sum over owned faces (descending) (rD_r upper) w_n
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_dic_rd(SolverParams sp, const double *__restrict__ diagB, const double *__restrict__ coef,
         const int32_t *__restrict__ row_start, const int32_t *__restrict__ col,
         const int32_t *__restrict__ owner_start, double *__restrict__ rD) {
    // red cells first need no lower faces; black cells read red diagonals only
    const CellRange cr = cell_range(sp.n, sp.chunk, logical_block());
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        double d = diagB[c];
        if (c >= sp.n_red) {
            const int32_t e_up = row_start[c + 1] - (owner_start[c + 1] - owner_start[c]);
            for (int32_t e = row_start[c]; e < e_up; ++e) {
                const double u = coef[e];
                d -= u * u / diagB[col[e]];
            }
        }
        rD[c] = 1.0 / d;
    }
}

// forward sweep on black rows, then (next kernel) backward sweep on red rows;
// each also accumulates its rows' share of w.r.
__global__ void __launch_bounds__(kBlock)
k_dic_forward(SolverParams sp, const double *__restrict__ coef, const int32_t *__restrict__ row_start,
              const int32_t *__restrict__ col, const int32_t *__restrict__ owner_start,
              const double *__restrict__ rD, const double *__restrict__ r, double *__restrict__ w,
              const PcgState *__restrict__ st) {
    if (load_state(st).done) return;
    const CellRange cr = cell_range(sp.n, sp.chunk, logical_block());
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        if (c < sp.n_red) continue;
        const double rd = rD[c];
        double wc = rd * r[c];
        const int32_t e_up = row_start[c + 1] - (owner_start[c + 1] - owner_start[c]);
        for (int32_t e = row_start[c]; e < e_up; ++e) {
            const int32_t o = col[e];
            wc -= rd * coef[e] * (rD[o] * r[o]);
        }
        w[c] = wc;
    }
}

__global__ void __launch_bounds__(kBlock)
k_dic_backward(SolverParams sp, const double *__restrict__ coef, const int32_t *__restrict__ row_start,
               const int32_t *__restrict__ col, const int32_t *__restrict__ owner_start,
               const double *__restrict__ rD, const double *__restrict__ r, double *__restrict__ w,
               double *__restrict__ part, const PcgState *__restrict__ st) {
    if (load_state(st).done) return;
    const int32_t L = logical_block();
    const CellRange cr = cell_range(sp.n, sp.chunk, L);
    double acc[1] = {0.0};
    for (int32_t c = cr.begin + threadIdx.x; c < cr.end; c += kBlock) {
        const double rc = r[c];
        double wc;
        if (c < sp.n_red) {
            const double rd = rD[c];
            wc = rd * rc;
            const int32_t e1 = row_start[c + 1];
            const int32_t e_up = e1 - (owner_start[c + 1] - owner_start[c]);
            for (int32_t e = e1 - 1; e >= e_up; --e) wc -= rd * coef[e] * w[col[e]];
            w[c] = wc;
        } else {
            wc = w[c];
        }
        acc[0] += wc * rc;
    }
    const int slots[1] = {kPartWr};
    write_partials<1>(part, slots, acc, L);
}

__global__ void k_any_nonfinite(const double *__restrict__ a, int32_t n, PcgState *st) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(&st->flag, 1);
}

__global__ void k_clear_flag(PcgState *st) { st->flag = 0; }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void carve_problem(Carver &cv, const lf_mesh *m, const lf_solver_opts &o, lf_problem *P) {
    const size_t N = m->N, F = m->F, B = m->B;
    auto *pt = cv.take<int32_t>(std::max<int32_t>(m->P, 1));
    auto *pv = cv.take<double>(std::max<int32_t>(m->P, 1));
    double *vec[11];
    for (auto &v : vec) v = cv.take<double>(N);
    auto *upper = cv.take<double>(F);
    auto *coef = cv.take<double>(2 * F);
    auto *ic = cv.take<double>(B);
    auto *bc = cv.take<double>(B);
    auto *part = cv.take<double>(static_cast<size_t>(kNumPart) * kMaxGrid);
    auto *state = cv.take<PcgState>(1);
    if (P) {
        P->patch_type = pt; P->patch_value = pv;
        P->T = vec[0]; P->r = vec[1]; P->p = vec[2]; P->q = vec[3]; P->w = vec[4]; P->rD = vec[5];
        P->sumA = vec[6]; P->diag = vec[7]; P->source = vec[8]; P->diagB = vec[9]; P->srcB = vec[10];
        P->upper = upper; P->coef = coef; P->int_coeff = ic; P->bou_coeff = bc; P->part = part;
        P->state = state;
    }
    if (o.precision == LF_PREC_MIXED) {
        auto *coef32 = cv.take<float>(2 * F);
        float *v32[6];
        for (auto &v : v32) v = cv.take<float>(N);
        if (P) {
            P->coef32 = coef32; P->diag32 = v32[0]; P->rD32 = v32[1]; P->r32 = v32[2];
            P->p32 = v32[3]; P->q32 = v32[4]; P->d32 = v32[5];
        }
    }
}

static inline dim3 cell_grid(const lf_problem *P) { return dim3(static_cast<unsigned>(P->grid.grid)); }

static lf_status launch_assemble(lf_problem *P, bool full, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    const double rdt = 1.0 / P->dt;
    if (full)
        LF_LAUNCH(P, LF_K_ASSEMBLE, s, k_assemble<true>, cell_grid(P), dim3(kBlock), 0, s, P->sp, rdt, P->DT, m->row_start,
                           m->face_of, m->owner_start, m->mag_sf, m->delta, m->bface_start, m->bface_list,
                           m->bface_patch, m->bmag_sf, m->bdelta, P->patch_type, P->patch_value, m->V, P->T,
                           P->coef, P->upper, P->diag, P->source, P->diagB, P->srcB, P->int_coeff,
                           P->bou_coeff);
    else
        LF_LAUNCH(P, LF_K_ASSEMBLE, s, k_assemble<false>, cell_grid(P), dim3(kBlock), 0, s, P->sp, rdt, P->DT, m->row_start,
                           m->face_of, m->owner_start, m->mag_sf, m->delta, m->bface_start, m->bface_list,
                           m->bface_patch, m->bmag_sf, m->bdelta, P->patch_type, P->patch_value, m->V, P->T,
                           P->coef, P->upper, P->diag, P->source, P->diagB, P->srcB, P->int_coeff,
                           P->bou_coeff);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

static lf_status launch_setup(lf_problem *P, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    const bool diag_pc = P->opts.precond == LF_PC_DIAGONAL;
    LF_LAUNCH(P, LF_K_SETUP1, s, k_setup1, cell_grid(P), dim3(kBlock), 0, s, P->sp, diag_pc ? 1 : 0, P->diagB, P->coef,
                       m->row_start, m->col, P->T, P->srcB, P->q, P->r, P->sumA, P->rD, P->part, P->state);
    if (!diag_pc) {
        LF_LAUNCH(P, LF_K_DIC_RD, s, k_dic_rd, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->diagB, P->coef, m->row_start,
                           m->col, m->owner_start, P->rD);
    }
    LF_LAUNCH(P, LF_K_SETUP2, s, k_setup2, cell_grid(P), dim3(kBlock), 0, s, P->sp, diag_pc ? 1 : 0, P->sumA, P->q,
                       P->srcB, P->rD, P->r, P->part);
    if (!diag_pc) {
        LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->coef, m->row_start, m->col,
                           m->owner_start, P->rD, P->r, P->w, P->state);
        LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->coef, m->row_start,
                           m->col, m->owner_start, P->rD, P->r, P->w, P->part, P->state);
    }
    LF_HIP(hipGetLastError());
    return LF_OK;
}

static void launch_direction(lf_problem *P, hipStream_t s) {
    if (P->opts.precond == LF_PC_DIAGONAL)
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction<true>, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->rD, P->r, P->w, P->p,
                           P->part, P->state);
    else
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction<false>, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->rD, P->r, P->w, P->p,
                           P->part, P->state);
}

// one PCG iteration after the direction update: q = A p, update, precondition,
// direction update of the next iteration (which also checks convergence)
static lf_status launch_iteration(lf_problem *P, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    const bool diag_pc = P->opts.precond == LF_PC_DIAGONAL;
    LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->diagB, P->coef, m->row_start,
                       m->col, P->p, P->q, P->part, P->state);
    if (diag_pc) {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update<true>, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->T, P->p, P->q, P->r, P->rD,
                           P->part, P->state);
    } else {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update<false>, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->T, P->p, P->q, P->r,
                           P->rD, P->part, P->state);
        LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->coef, m->row_start, m->col,
                           m->owner_start, P->rD, P->r, P->w, P->state);
        LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward, cell_grid(P), dim3(kBlock), 0, s, P->sp, P->coef, m->row_start,
                           m->col, m->owner_start, P->rD, P->r, P->w, P->part, P->state);
    }
    launch_direction(P, s);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

void prof_flush(lf_problem *P) {
    for (const auto &r : P->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            P->prof_ms[r.cls] += ms;
            P->prof_n[r.cls] += 1;
        }
    }
    P->prof_pending.clear();
    P->ev_used = 0;
}

static lf_status get_iter_graph(lf_problem *P, int lg) {
    if (P->g_iter[lg]) return LF_OK;
    if (!P->capture_stream) LF_HIP(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = P->capture_stream;
    LF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    lf_status st = LF_OK;
    for (int i = 0; i < (1 << lg) && st == LF_OK; ++i) st = launch_iteration(P, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != LF_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) { set_error("graph capture failed: %s", hipGetErrorString(e)); return LF_EDEVICE; }
    e = hipGraphInstantiate(&P->g_iter[lg], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { set_error("graph instantiate failed: %s", hipGetErrorString(e)); return LF_EDEVICE; }
    return LF_OK;
}

static lf_status launch_iterations(lf_problem *P, int32_t k) {
    hipStream_t s = P->stream;
    if (!P->opts.use_graph || P->prof_on) {
        for (int32_t i = 0; i < k; ++i) LF_TRY(launch_iteration(P, s));
        return LF_OK;
    }
    for (int lg = 6; lg >= 0; --lg) {
        while (k >= (1 << lg)) {
            LF_TRY(get_iter_graph(P, lg));
            LF_HIP(hipGraphLaunch(P->g_iter[lg], s));
            k -= 1 << lg;
        }
    }
    return LF_OK;
}

static lf_status solve_fp64(lf_problem *P, lf_solve_stats *out) {
    hipStream_t s = P->stream;
    LF_TRY(launch_setup(P, s));
    launch_direction(P, s);
    LF_HIP(hipGetLastError());
    const int32_t fixed_k = P->prof_on ? 1 : P->opts.iters_per_check;
    int32_t k = fixed_k > 0 ? fixed_k : std::max<int32_t>(1, P->last_iters > 0 ? P->last_iters : 8);
    int32_t launched = 0;
    for (;;) {
        k = std::min<int32_t>(k, std::max<int32_t>(1, P->sp.max_iter + 1 - launched));
        LF_TRY(launch_iterations(P, k));
        launched += k;
        LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        LF_HIP(hipEventRecord(P->ev[2], s));
        LF_HIP(hipEventSynchronize(P->ev[2]));
        prof_flush(P);
        if (P->h_state->done) break;
        if (launched > P->sp.max_iter + P->sp.min_iter + 8) {
            set_error("solver state never reached done after %d iterations", launched);
            return LF_ESTATE;
        }
        if (fixed_k <= 0) k = std::max<int32_t>(2, k / 2);
    }
    const PcgState &h = *P->h_state;
    out->initial_residual = h.res0;
    out->final_residual = h.res;
    out->n_iter = h.n_iter;
    out->converged = h.converged;
    out->singular = h.singular;
    out->nonfinite = h.nonfinite;
    out->n_outer = 1;
    return LF_OK;
}

}  // namespace lf

using namespace lf;

lf_status lf_solve_mixed(lf_problem *P, lf_solve_stats *out);   // lf_mixed.hip

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
    o->block_cells = 0;
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

lf_status lf_problem_create(const lf_mesh *m, const lf_patch_bc *bcs, double DT, double dt,
                            const lf_solver_opts *o, void *ws, size_t ws_bytes, void *stream, lf_problem **out) {
    clear_error();
    if (!out) { set_error("out is NULL"); return LF_EINVAL; }
    *out = nullptr;
    if (!m) { set_error("mesh is NULL"); return LF_EINVAL; }
    if (m->P > 0 && !bcs) { set_error("bcs is NULL"); return LF_EINVAL; }
    if (!(DT >= 0.0) || !std::isfinite(DT)) { set_error("DT must be finite and >= 0"); return LF_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be finite and > 0"); return LF_EINVAL; }
    lf_solver_opts opts;
    if (o) opts = *o; else lf_default_opts(&opts);
    if (opts.max_iter < 0 || opts.min_iter < 0 || !std::isfinite(opts.tol) || !std::isfinite(opts.rel_tol)) {
        set_error("bad solver options");
        return LF_EINVAL;
    }
    if (opts.precond != LF_PC_DIAGONAL && opts.precond != LF_PC_DIC) { set_error("unknown preconditioner"); return LF_EINVAL; }
    if (opts.precision != LF_PREC_FP64 && opts.precision != LF_PREC_MIXED) { set_error("unknown precision"); return LF_EINVAL; }
    if (opts.precond == LF_PC_DIC && m->F > 0 && !m->two_colour) {
        set_error("DIC needs a two-colour numbering (every owner < every neighbour)");
        return LF_EINVAL;
    }
    if (opts.precond == LF_PC_DIC && opts.precision == LF_PREC_MIXED) {
        set_error("the mixed-precision form uses the diagonal preconditioner");
        return LF_EINVAL;
    }
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
    P->grid = make_cell_grid(m->N, opts.block_cells);
    P->sp.tol = opts.tol;
    P->sp.rel_tol = opts.rel_tol;
    P->sp.max_iter = opts.max_iter;
    P->sp.min_iter = opts.min_iter;
    P->sp.n = m->N;
    P->sp.chunk = P->grid.chunk;
    P->sp.grid = P->grid.grid;
    P->sp.n_red = m->two_colour ? m->n_red : m->N;
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
    if (e == hipSuccess) e = hipMemsetAsync(P->part, 0, sizeof(double) * kNumPart * kMaxGrid, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) { set_error("problem setup failed: %s", hipGetErrorString(e)); return fail(LF_EDEVICE); }
    *out = P;
    return LF_OK;
}

lf_status lf_problem_destroy(lf_problem *P) {
    if (!P) return LF_OK;
    for (auto &g : P->g_iter) if (g) (void)hipGraphExecDestroy(g);
    if (P->g_prologue) (void)hipGraphExecDestroy(P->g_prologue);
    if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
    for (auto &e : P->ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : P->ev_pool) if (e) (void)hipEventDestroy(e);
    if (P->h_state) (void)hipHostFree(P->h_state);
    delete P;
    return LF_OK;
}

lf_status lf_set_T(lf_problem *P, const double *T, int32_t on_device) {
    clear_error();
    if (!P || !T) { set_error("NULL argument"); return LF_EINVAL; }
    const int32_t N = P->mesh->N;
    if (!on_device) {
        for (int32_t c = 0; c < N; ++c)
            if (!std::isfinite(T[c])) { set_error("T[%d] is not finite", c); return LF_EINVAL; }
        LF_HIP(hipMemcpyAsync(P->T, T, sizeof(double) * N, hipMemcpyHostToDevice, P->stream));
        LF_HIP(hipStreamSynchronize(P->stream));
        return LF_OK;
    }
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, P->stream, P->state);
    hipLaunchKernelGGL(k_any_nonfinite, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream, T, N, P->state);
    LF_HIP(hipGetLastError());
    LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, P->stream));
    LF_HIP(hipStreamSynchronize(P->stream));
    if (P->h_state->flag) { set_error("T holds a non-finite value"); return LF_EINVAL; }
    LF_HIP(hipMemcpyAsync(P->T, T, sizeof(double) * N, hipMemcpyDeviceToDevice, P->stream));
    return LF_OK;
}

lf_status lf_get_T(lf_problem *P, double *T, int32_t on_device) {
    clear_error();
    if (!P || !T) { set_error("NULL argument"); return LF_EINVAL; }
    const int32_t N = P->mesh->N;
    LF_HIP(hipMemcpyAsync(T, P->T, sizeof(double) * N, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          P->stream));
    if (!on_device) LF_HIP(hipStreamSynchronize(P->stream));
    return LF_OK;
}

lf_status lf_assemble(lf_problem *P) {
    clear_error();
    if (!P) { set_error("NULL problem"); return LF_EINVAL; }
    LF_TRY(launch_assemble(P, true, P->stream));
    P->assembled = true;
    return LF_OK;
}

lf_status lf_get_matrix(lf_problem *P, double *diag, double *upper, double *source, double *diag_b,
                        double *source_b, double *int_coeff, double *bou_coeff) {
    clear_error();
    if (!P) { set_error("NULL problem"); return LF_EINVAL; }
    if (!P->assembled) { set_error("call lf_assemble first"); return LF_ESTATE; }
    const lf_mesh *m = P->mesh;
    hipStream_t s = P->stream;
    const size_t N = m->N, F = m->F, B = m->B;
    if (diag) LF_HIP(hipMemcpyAsync(diag, P->diag, 8 * N, hipMemcpyDeviceToHost, s));
    if (source) LF_HIP(hipMemcpyAsync(source, P->source, 8 * N, hipMemcpyDeviceToHost, s));
    if (diag_b) LF_HIP(hipMemcpyAsync(diag_b, P->diagB, 8 * N, hipMemcpyDeviceToHost, s));
    if (source_b) LF_HIP(hipMemcpyAsync(source_b, P->srcB, 8 * N, hipMemcpyDeviceToHost, s));
    if (upper && F) LF_HIP(hipMemcpyAsync(upper, P->upper, 8 * F, hipMemcpyDeviceToHost, s));
    if (int_coeff && B) LF_HIP(hipMemcpyAsync(int_coeff, P->int_coeff, 8 * B, hipMemcpyDeviceToHost, s));
    if (bou_coeff && B) LF_HIP(hipMemcpyAsync(bou_coeff, P->bou_coeff, 8 * B, hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    return LF_OK;
}

lf_status lf_amul(lf_problem *P, const double *x, double *y) {
    clear_error();
    if (!P || !x || !y) { set_error("NULL argument"); return LF_EINVAL; }
    if (!P->assembled) { set_error("call lf_assemble first"); return LF_ESTATE; }
    const lf_mesh *m = P->mesh;
    hipLaunchKernelGGL(k_amul, cell_grid(P), dim3(kBlock), 0, P->stream, P->sp, P->diagB, P->coef, m->row_start,
                       m->col, x, y);
    LF_HIP(hipGetLastError());
    return LF_OK;
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

lf_status lf_step(lf_problem *P, int32_t n_steps, lf_solve_stats *stats) {
    clear_error();
    if (!P || n_steps < 0) { set_error("bad argument"); return LF_EINVAL; }
    hipStream_t s = P->stream;
    for (int32_t i = 0; i < n_steps; ++i) {
        lf_solve_stats st;
        std::memset(&st, 0, sizeof(st));
        LF_HIP(hipEventRecord(P->ev[0], s));
        LF_TRY(launch_assemble(P, false, s));
        LF_HIP(hipEventRecord(P->ev[1], s));
        P->assembled = true;
        if (P->opts.precision == LF_PREC_MIXED) {
            LF_TRY(lf_solve_mixed(P, &st));
        } else {
            LF_TRY(solve_fp64(P, &st));
        }
        float a_ms = 0.f, s_ms = 0.f;
        LF_HIP(hipEventElapsedTime(&a_ms, P->ev[0], P->ev[1]));
        LF_HIP(hipEventElapsedTime(&s_ms, P->ev[1], P->ev[2]));
        st.assemble_ms = a_ms;
        st.solve_ms = s_ms;
        P->last_iters = st.n_iter;
        if (stats) stats[i] = st;
        if (st.nonfinite) { set_error("non-finite residual in step %d", i); return LF_ENONFINITE; }
    }
    return LF_OK;
}

}  // extern "C"
