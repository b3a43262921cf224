// Per-step assembly of TEqn = ddt(T) - laplacian(DT, T) and its PCG solve.
//
// Cell-parallel kernels run one row per thread over the whole mesh (the
// hardware dispatcher balances workgroups over the CUs), gather through the
// sliced row layout (no atomics, so results are deterministic) and leave one
// partial sum per workgroup; one-workgroup kernels then sum the partials in a
// fixed order and take every scalar decision of the solver (step lengths,
// convergence, singularity), so the cell-parallel kernels only read the state.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "lf_solver.h"

namespace lf {

// kFull also stores diag/source without the boundary part (test hook).
// kSetup fuses the start of the PCG solve from x0 = T (the row's coefficients
// are at hand): wA = A x0, r = b - wA, the row sum of A, the row's terms
// |wA - pA| + |b - pA| of the normalisation factor (pA = row sum * mean(x0),
// the mean taken beforehand), and with the diagonal preconditioner
// rD = 1/diag, w.r and the first direction p = w; partial sums of |r|, those
// terms and w.r.  kMixed (precision form) instead starts the first refinement
// pass of the scaled inner system: s = sqrt(diag) rounded to FP32, the scaled
// residual rs = r / s rounded to FP32, y = 0, and the partial sums of s|rs|
// (the L1 norm of the residual the inner solve sees) and rs.rs.
// kNonorth (band meshes created non-orthogonal): the laplacian's explicit
// non-orthogonal source is computed here from the face records and the
// gradient (g, by component) instead of being read from a separate pass.

// The explicit non-orthogonal source of cell c on a band mesh: for each face,
// DT |S_f| k_f . (w g_P + (1 - w) g_N) with the face's owner-side weight,
// subtracted for the cell's lower faces (taken k = K-1 .. 0) and added for its
// owned faces (k = 0 .. K-1), the face loop's order; the sum divided by V and
// multiplied back, as the separate correction pass does term for term.  gk
// holds one record (k_x, k_y, k_z, w) per band slot.
template <int K>
__device__ __forceinline__ double band_nonorth_source(const BandLayout<K> &L, int32_t c, double DT, double v,
                                                      const double *__restrict__ g,
                                                      const double *__restrict__ gk) {
    const int64_t n = L.n;
    const double gc0 = g[c], gc1 = g[n + c], gc2 = g[2 * n + c];
    double div = 0.0;
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {      // lower faces (owner c - d_k): flux subtracted
        const bool ok = c >= L.d[k];
        const int64_t cl = ok ? c - L.d[k] : c;
        const int64_t slot = static_cast<int64_t>(k) * n + cl;
        const double mg = L.mag_sf[slot];
        const double2 qa = reinterpret_cast<const double2 *>(gk)[2 * slot];
        const double2 qb = reinterpret_cast<const double2 *>(gk)[2 * slot + 1];
        const double o0 = g[cl], o1 = g[n + cl], o2 = g[2 * n + cl];
        if (ok && mg > 0.0) {
            const double fx = qb.y * (o0 - gc0) + gc0;
            const double fy = qb.y * (o1 - gc1) + gc1;
            const double fz = qb.y * (o2 - gc2) + gc2;
            const double corr = qa.x * fx + qa.y * fy + qb.x * fz;
            div -= (DT * mg) * corr;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {           // owned faces (neighbour c + d_k): flux added
        const bool ok = c + static_cast<int64_t>(L.d[k]) < n;
        const int64_t cu = ok ? c + L.d[k] : c;
        const int64_t slot = static_cast<int64_t>(k) * n + c;
        const double mg = L.mag_sf[slot];
        const double2 qa = reinterpret_cast<const double2 *>(gk)[2 * slot];
        const double2 qb = reinterpret_cast<const double2 *>(gk)[2 * slot + 1];
        const double u0 = g[cu], u1 = g[n + cu], u2 = g[2 * n + cu];
        if (ok && mg > 0.0) {
            const double fx = qb.y * (gc0 - u0) + u0;
            const double fy = qb.y * (gc1 - u1) + u1;
            const double fz = qb.y * (gc2 - u2) + u2;
            const double corr = qa.x * fx + qa.y * fy + qb.x * fz;
            div += (DT * mg) * corr;
        }
    }
    div /= v;
    return 0.0 - v * div;
}

template <class Lay, bool kFull, bool kSetup, bool kMixed, bool kNonorth = false>
__device__ __forceinline__ void assemble_rows(
    int32_t blk, const SolverParams &sp, double rdt, double DT, const Lay &L, const int32_t *__restrict__ bface_start,
    const int32_t *__restrict__ bface_list, const int32_t *__restrict__ bface_patch,
    const double *__restrict__ bmag_sf, const double *__restrict__ bdelta, const int32_t *__restrict__ patch_type,
    const double *__restrict__ patch_value, const double *__restrict__ V, const double *__restrict__ T,
    double *__restrict__ coef, double *__restrict__ upper, double *__restrict__ diag, double *__restrict__ source,
    double *__restrict__ diagB, double *__restrict__ srcB, double *__restrict__ int_coeff,
    double *__restrict__ bou_coeff, int32_t diag_pc, double *__restrict__ r, double *__restrict__ rD,
    double *__restrict__ part, const PcgState *__restrict__ st, float *__restrict__ sig32, float *__restrict__ r32,
    float *__restrict__ d32, double *__restrict__ p, const double *__restrict__ lap_src,
    const double *__restrict__ T_old, const double *__restrict__ nb_g = nullptr,
    const double *__restrict__ nb_gk = nullptr, double *__restrict__ xs = nullptr) {
    const int32_t c = blk * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double x_avg = kSetup ? st->x_avg : 0.0;
    if (c < sp.n) {
        RowCoefs<Lay> rcf;
        const double lap_diag = assemble_coefs<kFull>(L, c, DT, coef, upper, rcf);
        const double v = V[c];
        const double d = rdt * v - lap_diag;
        const double xc = T[c];
        // TEqn = ddt - laplacian: the laplacian's explicit non-orthogonal
        // source (null on orthogonal meshes) is subtracted from the ddt source,
        // which uses T at the start of the step (T_old; null: T itself)
        const double xo = T_old ? T_old[c] : xc;
        double s;
        if constexpr (kNonorth)
            s = (rdt * xo) * v - band_nonorth_source(L, c, DT, v, nb_g, nb_gk);
        else
            s = lap_src ? (rdt * xo) * v - lap_src[c] : (rdt * xo) * v;
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
        if (kSetup) {
            double ax = db * xc, sa = db;
            row_amul_sum(L, c, coef, rcf, T, ax, sa);
            const double rc = sb - ax;
            const double pa = sa * x_avg;
            if (!kMixed && diag_pc != 2) r[c] = rc;
            acc[0] = fabs(rc);
            acc[1] = fabs(ax - pa) + fabs(sb - pa);
            if (diag_pc == 2 && !kMixed) {
                // the start of CG on the Jacobi-scaled system: r~ = r / sd, the
                // first direction p~ = r~, x~ = sd x0 (sd = sqrt(diagB), kept in
                // rD); w.r = r~.r~
                const double sd = sqrt(db);
                const double rt = rc / sd;
                rD[c] = sd;
                r[c] = rt;
                p[c] = rt;
                xs[c] = sd * xc;
                acc[2] = rt * rt;
            }
            if (diag_pc == 1 && !kMixed) {  // the precision form keeps only the FP32 rD
                const double rd = 1.0 / db;
                rD[c] = rd;
                const double wc = rd * rc;
                acc[2] = wc * rc;
                p[c] = wc;                  // first search direction p = w (used only if the solve iterates)
            }
            if (kMixed) {
                // start of the first refinement pass: rs = r / s rounded, y = 0
                const float sg32 = static_cast<float>(sqrt(db));
                const double sg = sg32;
                sig32[c] = sg32;
                const float rs = static_cast<float>(rc / sg);
                r32[c] = rs;
                d32[c] = 0.0f;
                acc[3] = fabs(sg * static_cast<double>(rs));
                acc[4] = static_cast<double>(rs) * static_cast<double>(rs);
            }
        }
    }
    if (kSetup && kMixed) {
        const int slots[5] = {kPartSumR, kPartNf, kPartWr, kPartSumR32, kPartWr32};
        write_partials_at<5>(part, sp.grid, blk, slots, acc);
    } else if (kSetup) {
        double a3[3] = {acc[0], acc[1], acc[2]};
        const int slots[3] = {kPartSumR, kPartNf, kPartWr};
        write_partials_at<3>(part, sp.grid, blk, slots, a3);
    }
}

template <class Lay, bool kFull, bool kSetup, bool kMixed, bool kNonorth = false>
__global__ void __launch_bounds__(kCellBlock)
k_assemble(SolverParams sp, double rdt, double DT, Lay L, const int32_t *__restrict__ bface_start,
           const int32_t *__restrict__ bface_list, const int32_t *__restrict__ bface_patch,
           const double *__restrict__ bmag_sf, const double *__restrict__ bdelta,
           const int32_t *__restrict__ patch_type, const double *__restrict__ patch_value,
           const double *__restrict__ V, const double *__restrict__ T, double *__restrict__ coef,
           double *__restrict__ upper, double *__restrict__ diag, double *__restrict__ source,
           double *__restrict__ diagB, double *__restrict__ srcB, double *__restrict__ int_coeff,
           double *__restrict__ bou_coeff, int32_t diag_pc, double *__restrict__ r, double *__restrict__ rD,
           double *__restrict__ part, const PcgState *__restrict__ st, float *__restrict__ sig32,
           float *__restrict__ r32, float *__restrict__ d32, double *__restrict__ p,
           const double *__restrict__ lap_src, const double *__restrict__ T_old,
           const double *__restrict__ nb_g, const double *__restrict__ nb_gk, double *__restrict__ xs) {
    assemble_rows<Lay, kFull, kSetup, kMixed, kNonorth>(
        static_cast<int32_t>(blockIdx.x), sp, rdt, DT, L, bface_start, bface_list, bface_patch, bmag_sf, bdelta,
        patch_type, patch_value, V, T, coef, upper, diag, source, diagB, srcB, int_coeff, bou_coeff, diag_pc, r, rD,
        part, st, sig32, r32, d32, p, lap_src, T_old, nb_g, nb_gk, xs);
}

// partial sums of x0 = T (its mean enters the normalisation factor)
__device__ __forceinline__ void sum_x_rows(int32_t blk, const SolverParams &sp, const double *__restrict__ T,
                                           double *__restrict__ part) {
    const int32_t c = blk * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {c < sp.n ? T[c] : 0.0};
    const int slots[1] = {kPartSumX};
    write_partials_at<1>(part, sp.grid, blk, slots, acc);
}

__global__ void __launch_bounds__(kCellBlock)
k_sum_x(SolverParams sp, const double *__restrict__ T, double *__restrict__ part) {
    sum_x_rows(static_cast<int32_t>(blockIdx.x), sp, T, part);
}

// y = A x (diag x first, then the row's entries in order)
template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_amul(SolverParams sp, Lay L, const double *__restrict__ diagB, const double *__restrict__ coef,
       const double *__restrict__ x, double *__restrict__ y) {
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) y[c] = layout_dot(L, c, coef, x, diagB[c] * x[c]);
}

// y = A x by the row walk (band layouts with two or more bands)
template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_amul_walk(BandLayout<K> L, const double *__restrict__ diagB, const double *__restrict__ coef,
            const double *__restrict__ x, double *__restrict__ y) {
    band_walk<K, false, false>(L, diagB, coef, x, y);
}

// y = A x by the block walk of a box
__global__ void __launch_bounds__(kBwBlock)
k_amul_box(BandLayout<3> L, BoxWalk bw, const double *__restrict__ diagB, const double *__restrict__ coef,
           const double *__restrict__ x, double *__restrict__ y) {
    typedef Lanes<double, 2> R;
    box_walk<double, 2, false, false>(L, bw, diagB, coef, x, [&](int64_t c, const R &yc, const R &, const R &) {
        y[c] = yc.v[0];
        y[c + 1] = yc.v[1];
    });
}

// band layout: face-order copy of the coefficients, upper_f at slot k*N + owner_f
__global__ void __launch_bounds__(kCellBlock)
k_band_upper(int32_t F, int32_t N, BandOffsets bo, const int32_t *__restrict__ owner,
             const int32_t *__restrict__ neighbour, const double *__restrict__ coef, double *__restrict__ upper) {
    const int64_t f = static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x;
    if (f >= F) return;
    const int32_t o = owner[f];
    const int32_t off = neighbour[f] - o;
    for (int32_t k = 0; k < bo.k; ++k)
        if (bo.d[k] == off) upper[f] = coef[static_cast<int64_t>(k) * N + o];
}

// Start of PCG iteration k: p = w (k = 0) or p = w + beta p, with w = rD r
// (diagonal) or the stored DIC residual.  For k > 0 the update
// x += alpha p of iteration k-1 is applied here, before p is overwritten
// (same operands and order as applying it at the end of iteration k-1).
template <bool kDiag>
__global__ void __launch_bounds__(kCellBlock)
k_direction(SolverParams sp, const double *__restrict__ rD, const double *__restrict__ r,
            const double *__restrict__ w, double *__restrict__ p, double *__restrict__ x,
            const PcgState *__restrict__ st) {
    if (st->done) return;
    const bool first = st->n_iter == 0;
    const double beta = st->beta, alpha = st->alpha;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) {
        const double wc = kDiag ? __builtin_nontemporal_load(&rD[c]) * r[c] : w[c];
        if (first) {
            p[c] = wc;
        } else {
            const double pc = p[c];
            // x is next needed an iteration later: stream it past the caches
            // that p, read by the product that follows, can use
            __builtin_nontemporal_store(__builtin_nontemporal_load(&x[c]) + alpha * pc, &x[c]);
            p[c] = wc + beta * pc;
        }
    }
}

// q = A p and the partial sums of q.p
template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_amul_dot(SolverParams sp, Lay L, const double *__restrict__ diagB, const double *__restrict__ coef,
           const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
           const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < sp.n) {
        const double pc = p[c];
        // diag and q are touched once per launch: stream them past the caches
        // that keep p and the coefficients for the neighbouring rows
        const double qc = layout_dot(L, c, coef, p, __builtin_nontemporal_load(&diagB[c]) * pc);
        __builtin_nontemporal_store(qc, &q[c]);
        acc[0] = qc * pc;
    }
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid, slots, acc);
}

// k_amul_dot by the row walk: sp.grid_amul workgroups, whose partials of q.p
// fill the first sp.grid_amul entries of the p.q slot (slots sp.grid apart)
template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_amul_dot_walk(SolverParams sp, BandLayout<K> L, const double *__restrict__ diagB, const double *__restrict__ coef,
                const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
                const PcgState *__restrict__ st) {
    if (st->done) return;
    double acc[1] = {band_walk<K, true, false>(L, diagB, coef, p, q)};
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid, slots, acc);
}

// k_amul_dot by the block walk of a box: bw.blocks workgroups of kBwBlock
// threads, whose partials of q.p fill the first bw.blocks entries of the p.q slot
__global__ void __launch_bounds__(kBwBlock)
k_amul_dot_box(SolverParams sp, BandLayout<3> L, BoxWalk bw, const double *__restrict__ diagB,
               const double *__restrict__ coef, const double *__restrict__ p, double *__restrict__ q,
               double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    double acc[1] = {0.0};
    typedef Lanes<double, 2> R;
    box_walk<double, 2, true, false>(L, bw, diagB, coef, p, [&](int64_t c, const R &qc, const R &pc, const R &) {
        lanes_store_stream(q, c, qc);
        acc[0] += qc.v[0] * pc.v[0];
        acc[0] += qc.v[1] * pc.v[1];
    });
    const int slots[1] = {kPartPq};
    write_partials<1, kBwBlock>(part, sp.grid, slots, acc);
}

// r -= alpha q; partial sums of |r| and (diagonal) of w.r, w = rD r.  With
// the diagonal preconditioner each thread takes kUpdRows rows (fewer partials
// for the reduction that follows: sp.grid_upd workgroups); with DIC one row,
// since the DIC sweep that follows writes the w.r partials on the cell grid.

template <bool kDiag>
__global__ void __launch_bounds__(kCellBlock)
k_update(SolverParams sp, const double *__restrict__ q, double *__restrict__ r, const double *__restrict__ rD,
         double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    constexpr int R = kDiag ? kUpdRows : 1;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t c = cell_row<R>(j);
        if (c >= sp.n) continue;
        const double rc = r[c] - alpha * __builtin_nontemporal_load(&q[c]);
        r[c] = rc;
        acc[0] += fabs(rc);
        if (kDiag) {
            const double wc = rD[c] * rc;
            acc[1] += wc * rc;
        }
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials<2>(part, sp.grid, slots, acc);
}

// ---------------------------------------------------------------------------
// Small solves with the diagonal preconditioner (at most kFoldPartials
// partials per slot): the decisions of k_finalize<kFinAlpha> and <kFinBeta>
// are taken inside the update and direction kernels, by every workgroup from
// the same partials in the same order, so all take the same one, and
// workgroup 0 records them in the state.  A state value that workgroup 0
// overwrites during a launch is read by the others from the copy the update
// made (wArA_prev, n_iter_prev, conv_prev); `done` is read once per workgroup,
// and a workgroup that already sees workgroup 0's new value takes the decision
// that value records.  Two dependent launches fewer per iteration, which is
// what an iteration costs on a small mesh.
// ---------------------------------------------------------------------------
// the state's done flag as one value for the whole workgroup
__device__ __forceinline__ bool group_done(const PcgState *__restrict__ st) {
    __shared__ int32_t s_done;
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    return s_done != 0;
}

// k_finalize<kFinAlpha> then k_update<true>
__global__ void __launch_bounds__(kCellBlock)
k_update_fold(SolverParams sp, const double *__restrict__ q, double *__restrict__ r, const double *__restrict__ rD,
              double *__restrict__ part, PcgState *__restrict__ st) {
    if (group_done(st)) return;
    double v[1];
    const int ps[1] = {kPartPq};
    reduce_partials<1, kCellBlock>(part, sp.grid, sp.grid_amul, ps, v);
    const double pq = v[0], wArA = st->wArA;
    const bool bad = !isfinite(pq), sing = !bad && fabs(pq) / st->nf < 1e-300;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (bad || sing) {
        if (lead) {
            if (bad)
                st->nonfinite = 1;
            else
                st->singular = 1;
            st->done = 1;
        }
        return;
    }
    const double alpha = wArA / pq;
    if (lead) {
        st->alpha = alpha;
        st->wArA_prev = wArA;
        st->n_iter_prev = st->n_iter;
        st->conv_prev = st->converged;
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kUpdRows; ++j) {
        const int32_t c = cell_row<kUpdRows>(j);
        if (c >= sp.n) continue;
        const double rc = r[c] - alpha * __builtin_nontemporal_load(&q[c]);
        r[c] = rc;
        acc[0] += fabs(rc);
        const double wc = rD[c] * rc;
        acc[1] += wc * rc;
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials<2>(part, sp.grid, slots, acc);
}

// k_finalize<kFinBeta> then k_direction<true> (never the first direction)
__global__ void __launch_bounds__(kCellBlock)
k_direction_fold(SolverParams sp, const double *__restrict__ rD, const double *__restrict__ r,
                 double *__restrict__ p, double *__restrict__ x, const double *__restrict__ part,
                 PcgState *__restrict__ st) {
    if (group_done(st)) return;
    double v[2];
    const int ps[2] = {kPartSumR, kPartWr};
    reduce_partials<2, kCellBlock>(part, sp.grid, sp.grid_upd, ps, v);
    const double res = v[0] / st->nf;
    const int32_t k = st->n_iter_prev + 1;
    const bool conv = (k < sp.max_iter) ? check_conv(res, st->res0, sp.tol, sp.rel_tol) : (st->conv_prev != 0);
    const bool cont = (k < sp.max_iter && !conv) || k < sp.min_iter;
    const bool bad = !isfinite(res) || !isfinite(v[1]);
    const double beta = v[1] / st->wArA_prev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->res = res;
        st->n_iter = k;
        st->converged = conv ? 1 : 0;
        if (bad) {
            st->nonfinite = 1;
            st->done = 1;
        } else if (!cont) {
            st->done = 1;
        } else {
            st->beta = beta;
            st->wArA = v[1];
        }
    }
    if (bad || !cont) return;
    const double alpha = st->alpha;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) {
        const double wc = __builtin_nontemporal_load(&rD[c]) * r[c];
        const double pc = p[c];
        __builtin_nontemporal_store(__builtin_nontemporal_load(&x[c]) + alpha * pc, &x[c]);
        p[c] = wc + beta * pc;
    }
}

// end of a solve: the update x += alpha p of the last counted iteration is
// still pending unless the solve stopped at a singular or non-finite point
// (then the pending update was applied by the last direction kernel).  The
// same launch writes k_sum_x's partial sums of the new x (same workgroups,
// same values), which the next solve's mean takes instead of a pass of its own.
__global__ void __launch_bounds__(kCellBlock)
k_commit(SolverParams sp, double *__restrict__ x, const double *__restrict__ p, double *__restrict__ part,
         const PcgState *__restrict__ st) {
    const bool apply = !(st->n_iter < 1 || st->singular || st->nonfinite);
    const double alpha = st->alpha;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < sp.n) {
        double xc = x[c];
        if (apply) {
            xc += alpha * p[c];
            x[c] = xc;
        }
        acc[0] = xc;
    }
    const int slots[1] = {kPartSumX};
    write_partials<1>(part, sp.grid, slots, acc);
}

// ---------------------------------------------------------------------------
// Diagonal FP64 solves on the block walk (not folded): CG on the Jacobi-scaled
// system.  With sd = sqrt(diagB) and S = diag(1/sd), the diagonally
// preconditioned CG of A (w = r / diagB) and plain CG on S A S, whose diagonal
// is 1, have the same iterates under x~ = sd x, r~ = r / sd, p~ = sd p,
// q~ = S A S p~ = q / sd: w.r = r~.r~, p.q = p~.q~, hence the same alpha and
// beta.  The assembly's set-up writes sd (into rD), r~, p~ = r~ and x~ (into
// w); the iteration's product then reads no diagonal and its direction update
// no reciprocal; the convergence test still takes the L1 norm of the residual
// of A, sum |sd r~|; the commit writes T = x~ / sd.
// ---------------------------------------------------------------------------

// coefficients of S A S in the band layout: slot k of row c holds
// a / (sd_c sd_{c+d_k}), 0 where the band has no face.  Two rows per thread;
// on every box with the block walk N, nx and nx ny are even (offsets 1, nx,
// nx ny), so the y and z neighbours' sd are 16-byte loads too, and row c's x
// neighbour is the thread's own row c + 1
__global__ void __launch_bounds__(kCellBlock)
k_scale_coef(BandLayout<3> L, const double *__restrict__ sd, const double *__restrict__ coef,
             double *__restrict__ coefS) {
    typedef Lanes<double, 2> R;
    const int64_t n = L.n;
    const int64_t c = 2 * (static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x);
    if (c >= n) return;
    const R s = lanes_load<double, 2>(sd, c);
    R sn[3];
    sn[0].v[0] = s.v[1];
    sn[0].v[1] = c + 2 < n ? sd[c + 2] : 1.0;
#pragma unroll
    for (int k = 1; k < 3; ++k) sn[k] = c + L.d[k] < n ? lanes_load<double, 2>(sd, c + L.d[k]) : s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t o = k * n + c;
        const R a = lanes_load<double, 2, true>(coef, o);
        R y;
#pragma unroll
        for (int w = 0; w < 2; ++w) y.v[w] = c + w + L.d[k] < n ? a.v[w] / (s.v[w] * sn[k].v[w]) : 0.0;
        lanes_store_stream(coefS, o, y);
    }
}

// q~ = (S A S) p~ and the partial sums of q~.p~ by the block walk
__global__ void __launch_bounds__(kBwBlock)
k_amul_dot_box_scaled(SolverParams sp, BandLayout<3> L, BoxWalk bw, const double *__restrict__ coefS,
                      const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
                      const PcgState *__restrict__ st) {
    if (st->done) return;
    double acc[1] = {0.0};
    typedef Lanes<double, 2> R;
    box_walk<double, 2, false, true>(L, bw, nullptr, coefS, p, [&](int64_t c, const R &qc, const R &pc, const R &) {
        lanes_store_stream(q, c, qc);
        acc[0] += qc.v[0] * pc.v[0];
        acc[0] += qc.v[1] * pc.v[1];
    });
    const int slots[1] = {kPartPq};
    write_partials<1, kBwBlock>(part, sp.grid, slots, acc);
}

// r~ -= alpha q~; partial sums of |sd r~| (the residual of A) and of r~.r~
// (w.r); kUpdRows rows per thread like k_update<true>, two adjacent rows per
// 16-byte access (N is even on every box with the block walk)
__global__ void __launch_bounds__(kCellBlock)
k_update_scaled(SolverParams sp, const double *__restrict__ q, double *__restrict__ r, const double *__restrict__ sd,
                double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    typedef Lanes<double, 2>::vec V;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kUpdRows / 2; ++j) {
        const int64_t c = 2 * static_cast<int64_t>(cell_row<kUpdRows / 2>(j));
        if (c >= sp.n) continue;
        const R qc = lanes_load<double, 2, true>(q, c);
        const R sc = lanes_load<double, 2, true>(sd, c);
        const R r0 = lanes_load<double, 2>(r, c);
        V y;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const double rc = r0.v[w] - alpha * qc.v[w];
            y[w] = rc;
            acc[0] += fabs(sc.v[w] * rc);
            acc[1] += rc * rc;
        }
        *reinterpret_cast<V *>(r + c) = y;
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials<2>(part, sp.grid, slots, acc);
}

// p~ = r~ + beta p~ with the deferred x~ += alpha p~ of the iteration before,
// as k_direction does for w = r~ (scaled solve): kUpdRows rows per thread,
// two adjacent rows per 16-byte access, on the update's grid
__global__ void __launch_bounds__(kCellBlock)
k_direction_scaled(SolverParams sp, const double *__restrict__ r, double *__restrict__ p, double *__restrict__ xs,
                   const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    typedef Lanes<double, 2>::vec V;
    const bool first = st->n_iter == 0;
    const double beta = st->beta, alpha = st->alpha;
#pragma unroll
    for (int j = 0; j < kUpdRows / 2; ++j) {
        const int64_t c = 2 * static_cast<int64_t>(cell_row<kUpdRows / 2>(j));
        if (c >= sp.n) continue;
        const R rc = lanes_load<double, 2>(r, c);
        V pn;
        if (first) {
#pragma unroll
            for (int w = 0; w < 2; ++w) pn[w] = rc.v[w];
        } else {
            const R pc = lanes_load<double, 2>(p, c);
            const R xc = lanes_load<double, 2, true>(xs, c);
            V xn;
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                xn[w] = xc.v[w] + alpha * pc.v[w];
                pn[w] = rc.v[w] + beta * pc.v[w];
            }
            // x~ is next needed an iteration later: past the caches
            __builtin_nontemporal_store(xn, reinterpret_cast<V *>(xs + c));
        }
        *reinterpret_cast<V *>(p + c) = pn;
    }
}

// end of a scaled solve: T = (x~ + alpha p~) / sd (the last pending update as
// in k_commit); T untouched when no iteration ran; partial sums of the new T
__global__ void __launch_bounds__(kCellBlock)
k_commit_scaled(SolverParams sp, double *__restrict__ T, const double *__restrict__ xs,
                const double *__restrict__ p, const double *__restrict__ sd, double *__restrict__ part,
                const PcgState *__restrict__ st) {
    const bool moved = st->n_iter >= 1;
    const bool apply = !(st->n_iter < 1 || st->singular || st->nonfinite);
    const double alpha = st->alpha;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < sp.n) {
        double tc;
        if (moved) {
            // x~, p~ and sd are not read again before the next solve writes them
            double xc = __builtin_nontemporal_load(&xs[c]);
            if (apply) xc += alpha * __builtin_nontemporal_load(&p[c]);
            tc = xc / __builtin_nontemporal_load(&sd[c]);
            T[c] = tc;
        } else {
            tc = T[c];
        }
        acc[0] = tc;
    }
    const int slots[1] = {kPartSumX};
    write_partials<1>(part, sp.grid, slots, acc);
}

// ---------------------------------------------------------------------------
// DIC on a two-colour numbering (cells [0, n_red) red, [n_red, N) black; every
// face has a red owner and a black neighbour, so a red row holds only owned
// faces and a black row only lower faces).  The sequential DIC recurrences
// then become cell-parallel gathers in the same order:
//   rD_red = diag, rD_black = diag - sum over its lower faces (ascending) of
//   upper^2 / rD_owner;  rD = 1/rD.
//   forward:  w_b = rD_b r_b - sum over lower faces (ascending) (rD_b upper) w_o
//             with w_o = rD_o r_o for the red owners
//   backward: w_r = rD_r r_r - sum over owned faces (descending) (rD_r upper) w_n
// ---------------------------------------------------------------------------
// a black row's DIC diagonal with slice width W: loads first, then the terms in
// ascending entry order (padding entries loaded, never used)
template <int W>
__device__ __forceinline__ double dic_rd_row(int32_t base, int32_t len, const MeshRows &mr,
                                             const double *__restrict__ coef, const double *__restrict__ diagB,
                                             double d) {
    int32_t col[W];
    double a[W], dg[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        col[j] = mr.scol[base + kSlice * j];
        a[j] = coef[base + kSlice * j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j) dg[j] = diagB[col[j]];
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (j < len) d -= a[j] * a[j] / dg[j];
    return d;
}

__global__ void __launch_bounds__(kCellBlock)
k_dic_rd(SolverParams sp, MeshRows mr, const double *__restrict__ diagB, const double *__restrict__ coef,
         double *__restrict__ rD) {
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c >= sp.n) return;
    double d = diagB[c];
    if (c >= sp.n_red) {
        const int32_t s = c >> 6;
        const int32_t base = mr.soff[s] + (c & (kSlice - 1));
        const int32_t width = (mr.soff[s + 1] - mr.soff[s]) >> 6;
        const int32_t len = mr.rlen[c];
        switch (width) {
            case 0: break;
            case 1: d = dic_rd_row<1>(base, len, mr, coef, diagB, d); break;
            case 2: d = dic_rd_row<2>(base, len, mr, coef, diagB, d); break;
            case 3: d = dic_rd_row<3>(base, len, mr, coef, diagB, d); break;
            case 4: d = dic_rd_row<4>(base, len, mr, coef, diagB, d); break;
            case 5: d = dic_rd_row<5>(base, len, mr, coef, diagB, d); break;
            case 6: d = dic_rd_row<6>(base, len, mr, coef, diagB, d); break;
            default: {
                int32_t idx = base;
                for (int32_t j = 0; j < len; ++j, idx += kSlice) {
                    const double u = coef[idx];
                    d -= u * u / diagB[mr.scol[idx]];
                }
            }
        }
    }
    rD[c] = 1.0 / d;
}

// A sweep row with slice width W: every entry's column and coefficient (read
// once per sweep: streamed past the caches) and its gathered operands are
// loaded first, then the terms are taken in the recurrence's order (forward:
// ascending entries; backward: descending).  Padding entries (j >= len) point
// at the row itself; they are loaded, never used.
template <int W>
__device__ __forceinline__ double dic_forward_row(int32_t base, int32_t len, const MeshRows &mr,
                                                  const double *__restrict__ coef, const double *__restrict__ rD,
                                                  const double *__restrict__ r, double rd, double wc) {
    int32_t col[W];
    double a[W], ro[W], rdo[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        col[j] = __builtin_nontemporal_load(&mr.scol[base + kSlice * j]);
        a[j] = __builtin_nontemporal_load(&coef[base + kSlice * j]);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        rdo[j] = rD[col[j]];
        ro[j] = r[col[j]];
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (j < len) wc -= rd * a[j] * (rdo[j] * ro[j]);
    return wc;
}

template <int W>
__device__ __forceinline__ double dic_backward_row(int32_t base, int32_t len, const MeshRows &mr,
                                                   const double *__restrict__ coef, const double *__restrict__ w,
                                                   double rd, double wc) {
    int32_t col[W];
    double a[W], wo[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        col[j] = __builtin_nontemporal_load(&mr.scol[base + kSlice * j]);
        a[j] = __builtin_nontemporal_load(&coef[base + kSlice * j]);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) wo[j] = w[col[j]];
#pragma unroll
    for (int j = W - 1; j >= 0; --j)
        if (j < len) wc -= rd * a[j] * wo[j];
    return wc;
}

__global__ void __launch_bounds__(kCellBlock)
k_dic_forward(SolverParams sp, MeshRows mr, const double *__restrict__ coef, const double *__restrict__ rD,
              const double *__restrict__ r, double *__restrict__ w, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c >= sp.n || c < sp.n_red) return;
    const double rd = rD[c];
    double wc = rd * r[c];
    const int32_t s = c >> 6;
    const int32_t base = mr.soff[s] + (c & (kSlice - 1));
    const int32_t width = (mr.soff[s + 1] - mr.soff[s]) >> 6;
    const int32_t len = mr.rlen[c];
    switch (width) {
        case 0: break;
        case 1: wc = dic_forward_row<1>(base, len, mr, coef, rD, r, rd, wc); break;
        case 2: wc = dic_forward_row<2>(base, len, mr, coef, rD, r, rd, wc); break;
        case 3: wc = dic_forward_row<3>(base, len, mr, coef, rD, r, rd, wc); break;
        case 4: wc = dic_forward_row<4>(base, len, mr, coef, rD, r, rd, wc); break;
        case 5: wc = dic_forward_row<5>(base, len, mr, coef, rD, r, rd, wc); break;
        case 6: wc = dic_forward_row<6>(base, len, mr, coef, rD, r, rd, wc); break;
        default: {
            int32_t idx = base;
            for (int32_t j = 0; j < len; ++j, idx += kSlice) {
                const int32_t o = mr.scol[idx];
                wc -= rd * coef[idx] * (rD[o] * r[o]);
            }
        }
    }
    w[c] = wc;
}

// backward sweep on red rows; all rows contribute their w.r partial
__global__ void __launch_bounds__(kCellBlock)
k_dic_backward(SolverParams sp, MeshRows mr, const double *__restrict__ coef, const double *__restrict__ rD,
               const double *__restrict__ r, double *__restrict__ w, double *__restrict__ part,
               const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < sp.n) {
        const double rc = r[c];
        double wc;
        if (c < sp.n_red) {
            const double rd = rD[c];
            wc = rd * rc;
            const int32_t s = c >> 6;
            const int32_t base = mr.soff[s] + (c & (kSlice - 1));
            const int32_t width = (mr.soff[s + 1] - mr.soff[s]) >> 6;
            const int32_t len = mr.rlen[c];
            switch (width) {
                case 0: break;
                case 1: wc = dic_backward_row<1>(base, len, mr, coef, w, rd, wc); break;
                case 2: wc = dic_backward_row<2>(base, len, mr, coef, w, rd, wc); break;
                case 3: wc = dic_backward_row<3>(base, len, mr, coef, w, rd, wc); break;
                case 4: wc = dic_backward_row<4>(base, len, mr, coef, w, rd, wc); break;
                case 5: wc = dic_backward_row<5>(base, len, mr, coef, w, rd, wc); break;
                case 6: wc = dic_backward_row<6>(base, len, mr, coef, w, rd, wc); break;
                default: {
                    int32_t idx = base + (len - 1) * kSlice;
                    for (int32_t j = len - 1; j >= 0; --j, idx -= kSlice) wc -= rd * coef[idx] * w[mr.scol[idx]];
                }
            }
            w[c] = wc;
        } else {
            wc = w[c];
        }
        acc[0] = wc * rc;
    }
    const int slots[1] = {kPartWr};
    write_partials<1>(part, sp.grid, slots, acc);
}

// ---------------------------------------------------------------------------
// The same DIC on the two-colour band layout: the same recurrences and term
// order, entries from rb_row (absent faces skipped).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCellBlock)
k_dic_rd_rb(SolverParams sp, RBLayout L, const double *__restrict__ diagB, const double *__restrict__ coef,
            double *__restrict__ rD) {
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c >= sp.n) return;
    double d = diagB[c];
    if (c >= sp.n_red) {
        int64_t slot[6];
        int32_t col[6];
        bool ok[6];
        rb_row(L.f, c, slot, col, ok);
        double a[6], dg[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            a[j] = coef[slot[j]];
            dg[j] = diagB[col[j]];
        }
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (ok[j]) d -= a[j] * a[j] / dg[j];
    }
    rD[c] = 1.0 / d;
}

__global__ void __launch_bounds__(kCellBlock)
k_dic_forward_rb(SolverParams sp, RBLayout L, const double *__restrict__ coef, const double *__restrict__ rD,
                 const double *__restrict__ r, double *__restrict__ w, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = sp.n_red + static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c >= sp.n) return;
    const double rd = rD[c];
    double wc = rd * r[c];
    int64_t slot[6];
    int32_t col[6];
    bool ok[6];
    rb_row(L.f, c, slot, col, ok);
    double a[6], ro[6], rdo[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        a[j] = coef[slot[j]];
        rdo[j] = rD[col[j]];
        ro[j] = r[col[j]];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if (ok[j]) wc -= rd * a[j] * (rdo[j] * ro[j]);
    w[c] = wc;
}

// The same forward sweep fused with the iteration's update of r on the
// two-colour band layout (one thread per red-black pair, sp.grid_amul
// workgroups): the black row's r -= alpha q is written here, the red rows' by
// the backward sweep that follows, so the red neighbours' updated r (the
// value the separate update would have stored, the same expression) is formed
// here from the old r and q.  Partial sums of the black rows' |r| go to the
// |r| slot; the backward sweep adds the red rows' to them.
__global__ void __launch_bounds__(kCellBlock)
k_dic_update_forward_rb(SolverParams sp, RBLayout L, const double *__restrict__ coef,
                        const double *__restrict__ rD, const double *__restrict__ q, double *__restrict__ r,
                        double *__restrict__ w, double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t nr = L.f.nr;
    const double alpha = st->alpha;
    const int32_t u = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (u < nr) {
        const int32_t c = nr + u;
        const double rc = r[c] - alpha * __builtin_nontemporal_load(&q[c]);
        r[c] = rc;
        acc[0] = fabs(rc);
        const double rd = rD[c];
        double wc = rd * rc;
        int64_t slot[6];
        int32_t col[6];
        bool ok[6];
        rb_row(L.f, c, slot, col, ok);
        double a[6], ro[6], rdo[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            a[j] = coef[slot[j]];
            rdo[j] = rD[col[j]];
            ro[j] = r[col[j]] - alpha * q[col[j]];
        }
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (ok[j]) wc -= rd * a[j] * (rdo[j] * ro[j]);
        w[c] = wc;
    }
    const int slots[1] = {kPartSumR};
    write_partials<1>(part, sp.grid, slots, acc);
}

// backward sweep on red rows; every row contributes its w.r partial
__global__ void __launch_bounds__(kCellBlock)
k_dic_backward_rb(SolverParams sp, RBLayout L, const double *__restrict__ coef, const double *__restrict__ rD,
                  const double *__restrict__ r, double *__restrict__ w, double *__restrict__ part,
                  const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < sp.n) {
        const double rc = r[c];
        double wc;
        if (c < sp.n_red) {
            const double rd = rD[c];
            wc = rd * rc;
            int64_t slot[6];
            int32_t col[6];
            bool ok[6];
            rb_row(L.f, c, slot, col, ok);
            double a[6], wo[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                a[j] = coef[slot[j]];
                wo[j] = w[col[j]];
            }
#pragma unroll
            for (int j = 5; j >= 0; --j)
                if (ok[j]) wc -= rd * a[j] * wo[j];
            w[c] = wc;
        } else {
            wc = w[c];
        }
        acc[0] = wc * rc;
    }
    const int slots[1] = {kPartWr};
    write_partials<1>(part, sp.grid, slots, acc);
}

// q = A p on the two-colour band layout, one thread per half-index u taking
// the red row u and the black row nr + u (x-neighbours on the box, so the
// coefficients a black row gathers from its red neighbours' slots are read
// near the time the red rows read them); partial sums of p.q over the pairs
// (sp.grid_amul workgroups)
__global__ void __launch_bounds__(kCellBlock)
k_amul_dot_rb(SolverParams sp, RBLayout L, const double *__restrict__ diagB, const double *__restrict__ coef,
              const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
              const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t nr = L.f.nr;
    const int32_t u = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (u < nr) {
        int64_t rs[6], bs[6];
        int32_t rc[6], bc[6];
        bool rok[6], bok[6];
        rb_pair(L.f, u, rs, rc, rok, bs, bc, bok);
        double ra[6], rx[6], ba[6], bx[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double v = coef[rs[j]], w = coef[bs[j]];
            ra[j] = rok[j] ? v : 0.0;
            ba[j] = bok[j] ? w : 0.0;
            rx[j] = p[rc[j]];
            bx[j] = p[bc[j]];
        }
        const double pr = p[u], pb = p[nr + u];
        double qr = __builtin_nontemporal_load(&diagB[u]) * pr;
        double qb = __builtin_nontemporal_load(&diagB[nr + u]) * pb;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            qr += ra[j] * rx[j];
            qb += ba[j] * bx[j];
        }
        __builtin_nontemporal_store(qr, &q[u]);
        __builtin_nontemporal_store(qb, &q[nr + u]);
        acc[0] = qr * pr + qb * pb;
    }
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid, slots, acc);
}

// q = A p on the two-colour band layout, two red-black pairs per lane
// (rb2_product; sp.grid_amul workgroups), with partial sums of p.q
__global__ void __launch_bounds__(kCellBlock)
k_amul_dot_rb2(SolverParams sp, RBLayout L, const double *__restrict__ diagB, const double *__restrict__ coef,
               const double *__restrict__ p, double *__restrict__ q, double *__restrict__ part,
               const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    const int64_t nr = L.f.nr;
    double acc[1] = {0.0};
    rb2_product(L.f, diagB, coef, p, [&](int64_t u, const R &qr, const R &qb, const R &pr, const R &pb) {
        lanes_store_stream(q, u, qr);
        lanes_store_stream(q, nr + u, qb);
        acc[0] += qr.v[0] * pr.v[0] + qb.v[0] * pb.v[0];
        acc[0] += qr.v[1] * pr.v[1] + qb.v[1] * pb.v[1];
    });
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid, slots, acc);
}

// the product alone (test hook)
__global__ void __launch_bounds__(kCellBlock)
k_amul_rb2(RBLayout L, const double *__restrict__ diagB, const double *__restrict__ coef,
           const double *__restrict__ x, double *__restrict__ y) {
    typedef Lanes<double, 2> R;
    const int64_t nr = L.f.nr;
    rb2_product(L.f, diagB, coef, x, [&](int64_t u, const R &qr, const R &qb, const R &, const R &) {
        y[u] = qr.v[0];
        y[u + 1] = qr.v[1];
        y[nr + u] = qb.v[0];
        y[nr + u + 1] = qb.v[1];
    });
}

// The assembly on the two-colour band layout with two red-black pairs per lane
// (the lanes of k_amul_dot_rb2; orthogonal meshes, T_old not used): a red
// row's six slot factors (delta, |S|) are 16-byte loads of its own slots, a
// black row's are its red neighbours' mirrored slots (one line or plane away,
// the lane's red pair, or the adjacent lane's), and the neighbours' x0 = T
// likewise; each row's coefficients, lapDiag, boundary fold and (kSetup) A x0,
// residual and normalisation terms come from the one-row kernel's expressions
// in its order, so the matrix is bitwise the same.  kSetup: the partial sums
// per workgroup, and zeros in each slot's further entries up to the cell
// grid's count (the reduction that follows reads that many).
template <bool kFull, bool kSetup>
__global__ void __launch_bounds__(kCellBlock)
k_assemble_rb2(SolverParams sp, double rdt, double DT, RBLayout L, const int32_t *__restrict__ bface_start,
               const int32_t *__restrict__ bface_list, const int32_t *__restrict__ bface_patch,
               const double *__restrict__ bmag_sf, const double *__restrict__ bdelta,
               const int32_t *__restrict__ patch_type, const double *__restrict__ patch_value,
               const double *__restrict__ V, const double *__restrict__ T, double *__restrict__ coef,
               double *__restrict__ diag, double *__restrict__ source, double *__restrict__ diagB,
               double *__restrict__ srcB, double *__restrict__ int_coeff, double *__restrict__ bou_coeff,
               double *__restrict__ r, double *__restrict__ part, const PcgState *__restrict__ st) {
    typedef Lanes<double, 2> R;
    typedef typename R::vec RV;
    const RBForm &f = L.f;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    const Rb2Lane l = rb2_lane(f);
    const int64_t u = l.u, pos = l.pos;
    const int32_t par = l.par;
    const R z = lanes_zero<double, 2>();
    const double x_avg = kSetup ? st->x_avg : 0.0;
    R dl[6], ms[6], tr = z, tb = z;
#pragma unroll
    for (int j = 0; j < 6; ++j) dl[j] = ms[j] = z;
    if (l.tv) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            dl[j] = lanes_load<double, 2>(L.delta, j * nr + u);
            ms[j] = lanes_load<double, 2>(L.mag_sf, j * nr + u);
        }
        tr = lanes_load<double, 2>(T, u);
        tb = lanes_load<double, 2>(T, nr + u);
    }
    // the adjacent lanes': slot +x factors and T at u - 1, slot -x factors and T at u + 2
    double d3m = lane_from_below(dl[3].v[1]), m3m = lane_from_below(ms[3].v[1]);
    double tbm = lane_from_below(tb.v[1]), trm = lane_from_below(tr.v[1]);
    double d2p = lane_from_above(dl[2].v[0]), m2p = lane_from_above(ms[2].v[0]);
    double tbp = lane_from_above(tb.v[0]), trp = lane_from_above(tr.v[0]);
    double acc[3] = {0.0, 0.0, 0.0};
    if (l.tv) {
        if (!l.below_ok && pos >= 2) {
            d3m = L.delta[3 * nr + u - 1];
            m3m = L.mag_sf[3 * nr + u - 1];
            tbm = T[nr + u - 1];
            trm = T[u - 1];
        }
        if (!l.above_ok && pos + 2 <= h - 1) {
            d2p = L.delta[2 * nr + u + 2];
            m2p = L.mag_sf[2 * nr + u + 2];
            tbp = T[nr + u + 2];
            trp = T[u + 2];
        }
        // one plane down, one line down, one line up, one plane up: the red
        // neighbours' mirrored slots (+z, +y, -y, -z) and T of both colours
        const int64_t off[4] = {-H, -h, h, H};
        const int slot[4] = {5, 4, 1, 0};
        const bool has[4] = {l.zlo, l.ylo, l.yhi, l.zhi};
        R ndl[4], nms[4], ntb[4], ntr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ndl[i] = nms[i] = ntb[i] = ntr[i] = z;
            if (has[i]) {
                const int64_t v = u + off[i];
                ndl[i] = lanes_load<double, 2>(L.delta, slot[i] * nr + v);
                nms[i] = lanes_load<double, 2>(L.mag_sf, slot[i] * nr + v);
                ntb[i] = lanes_load<double, 2>(T, nr + v);
                ntr[i] = lanes_load<double, 2>(T, v);
            }
        }
        const R vr = lanes_load<double, 2>(V, u), vb = lanes_load<double, 2>(V, nr + u);
        R ca[6], dd[2], ss[2], dbv[2], sbv[2], rv[2];
        // q = 0: the red rows u, u + 1; q = 1: the black rows nr + u, nr + u + 1
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t pk = pos + k;
                const int64_t c = (q == 0 ? 0 : nr) + u + k;
                bool ok[6];
                double fd[6], fm[6], xv[6];
                const double own = q == 0 ? tb.v[k] : tr.v[k];   // x of an absent entry
                if (q == 0) {
                    const bool o6[6] = {l.zlo, l.ylo, pk + par - 1 >= 0, pk + par <= h - 1, l.yhi, l.zhi};
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        ok[j] = o6[j];
                        fd[j] = dl[j].v[k];
                        fm[j] = ms[j].v[k];
                    }
                    xv[0] = ntb[0].v[k];
                    xv[1] = ntb[1].v[k];
                    xv[2] = par ? tb.v[k] : (k == 0 ? tbm : tb.v[0]);
                    xv[3] = par ? (k == 0 ? tb.v[1] : tbp) : tb.v[k];
                    xv[4] = ntb[2].v[k];
                    xv[5] = ntb[3].v[k];
                } else {
                    const bool o6[6] = {l.zlo, l.ylo, pk >= par, pk + 1 - par <= h - 1, l.yhi, l.zhi};
#pragma unroll
                    for (int j = 0; j < 6; ++j) ok[j] = o6[j];
                    fd[0] = ndl[0].v[k];
                    fm[0] = nms[0].v[k];
                    fd[1] = ndl[1].v[k];
                    fm[1] = nms[1].v[k];
                    fd[2] = par ? (k == 0 ? d3m : dl[3].v[0]) : dl[3].v[k];
                    fm[2] = par ? (k == 0 ? m3m : ms[3].v[0]) : ms[3].v[k];
                    fd[3] = par ? dl[2].v[k] : (k == 0 ? dl[2].v[1] : d2p);
                    fm[3] = par ? ms[2].v[k] : (k == 0 ? ms[2].v[1] : m2p);
                    fd[4] = ndl[2].v[k];
                    fm[4] = nms[2].v[k];
                    fd[5] = ndl[3].v[k];
                    fm[5] = nms[3].v[k];
                    xv[0] = ntr[0].v[k];
                    xv[1] = ntr[1].v[k];
                    xv[2] = par ? (k == 0 ? trm : tr.v[0]) : tr.v[k];
                    xv[3] = par ? tr.v[k] : (k == 0 ? tr.v[1] : trp);
                    xv[4] = ntr[2].v[k];
                    xv[5] = ntr[3].v[k];
                }
                double a[6], lap_diag = 0.0;
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    const double dlj = ok[j] ? fd[j] : 0.0, msj = ok[j] ? fm[j] : 0.0;
                    const double lap_upper = dlj * (DT * msj);
                    a[j] = -lap_upper;
                    lap_diag -= lap_upper;
                    if (!ok[j]) xv[j] = own;
                }
                if (q == 0) {
#pragma unroll
                    for (int j = 0; j < 6; ++j) ca[j].v[k] = a[j];
                }
                const double vv = q == 0 ? vr.v[k] : vb.v[k];
                const double xc = q == 0 ? tr.v[k] : tb.v[k];
                const double d = rdt * vv - lap_diag;
                const double src = (rdt * xc) * vv;
                double db = d, sb = src;
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
                dd[q].v[k] = d;
                ss[q].v[k] = src;
                dbv[q].v[k] = db;
                sbv[q].v[k] = sb;
                if (kSetup) {
                    double ax = db * xc, sa = db;
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        ax += a[j] * xv[j];
                        sa += a[j];
                    }
                    const double rc = sb - ax;
                    const double pa = sa * x_avg;
                    rv[q].v[k] = rc;
                    acc[0] += fabs(rc);
                    acc[1] += fabs(ax - pa) + fabs(sb - pa);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) *reinterpret_cast<RV *>(coef + j * nr + u) = RV{ca[j].v[0], ca[j].v[1]};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t c0 = (q == 0 ? 0 : nr) + u;
            if (kFull) {
                *reinterpret_cast<RV *>(diag + c0) = RV{dd[q].v[0], dd[q].v[1]};
                *reinterpret_cast<RV *>(source + c0) = RV{ss[q].v[0], ss[q].v[1]};
            }
            *reinterpret_cast<RV *>(diagB + c0) = RV{dbv[q].v[0], dbv[q].v[1]};
            *reinterpret_cast<RV *>(srcB + c0) = RV{sbv[q].v[0], sbv[q].v[1]};
            if (kSetup) *reinterpret_cast<RV *>(r + c0) = RV{rv[q].v[0], rv[q].v[1]};
        }
    }
    if (kSetup) {
        const int slots[3] = {kPartSumR, kPartNf, kPartWr};
        write_partials<3>(part, sp.grid, slots, acc);
        if (threadIdx.x == 0)
            for (int64_t j = gridDim.x + static_cast<int64_t>(blockIdx.x); j < sp.grid; j += gridDim.x)
#pragma unroll
                for (int q = 0; q < 3; ++q) part[static_cast<int64_t>(slots[q]) * sp.grid + j] = 0.0;
    }
}

// k_dic_rd_rb with two red-black pairs per lane: red rows 1/diag, black rows
// 1/(diag - sum over their red neighbours, in the row's order, of a^2 / the
// neighbour's diag), neighbours as in k_dic_forward_rb2
__global__ void __launch_bounds__(kCellBlock)
k_dic_rd_rb2(RBLayout L, const double *__restrict__ diagB, const double *__restrict__ coef,
             double *__restrict__ rD) {
    typedef Lanes<double, 2> R;
    const RBForm &f = L.f;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    const Rb2Lane l = rb2_lane(f);
    const int64_t u = l.u, pos = l.pos;
    const int32_t par = l.par;
    const R z = lanes_zero<double, 2>();
    R dr = z, s2 = z, s3 = z;
    if (l.tv) {
        dr = lanes_load<double, 2>(diagB, u);
        s2 = lanes_load<double, 2>(coef, 2 * nr + u);
        s3 = lanes_load<double, 2>(coef, 3 * nr + u);
    }
    double d_m1 = lane_from_below(dr.v[1]), s3_m1 = lane_from_below(s3.v[1]);
    double d_p2 = lane_from_above(dr.v[0]), s2_p2 = lane_from_above(s2.v[0]);
    if (!l.tv) return;
    if (!l.below_ok && pos >= 2) {
        d_m1 = diagB[u - 1];
        s3_m1 = coef[3 * nr + u - 1];
    }
    if (!l.above_ok && pos + 2 <= h - 1) {
        d_p2 = diagB[u + 2];
        s2_p2 = coef[2 * nr + u + 2];
    }
    const int64_t off[4] = {-H, -h, h, H};
    const int slot[4] = {5, 4, 1, 0};
    const bool has[4] = {l.zlo, l.ylo, l.yhi, l.zhi};
    R nd[4], nsl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        nd[i] = nsl[i] = z;
        if (has[i]) {
            nd[i] = lanes_load<double, 2>(diagB, u + off[i]);
            nsl[i] = lanes_load<double, 2>(coef, slot[i] * nr + u + off[i]);
        }
    }
    const R db = lanes_load<double, 2>(diagB, nr + u);
    R rr, rb;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int64_t pk = pos + k;
        rr.v[k] = 1.0 / dr.v[k];
        const double a2 = par ? (k == 0 ? s3_m1 : s3.v[0]) : s3.v[k];
        const double g2 = par ? (k == 0 ? d_m1 : dr.v[0]) : dr.v[k];
        const double a3 = par ? s2.v[k] : (k == 0 ? s2.v[1] : s2_p2);
        const double g3 = par ? dr.v[k] : (k == 0 ? dr.v[1] : d_p2);
        const bool ok[6] = {l.zlo, l.ylo, pk >= par, pk + 1 - par <= h - 1, l.yhi, l.zhi};
        const double a[6] = {nsl[0].v[k], nsl[1].v[k], a2, a3, nsl[2].v[k], nsl[3].v[k]};
        const double dg[6] = {nd[0].v[k], nd[1].v[k], g2, g3, nd[2].v[k], nd[3].v[k]};
        double d = db.v[k];
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (ok[j]) d -= a[j] * a[j] / dg[j];
        rb.v[k] = 1.0 / d;
    }
    *reinterpret_cast<typename R::vec *>(rD + u) = typename R::vec{rr.v[0], rr.v[1]};
    *reinterpret_cast<typename R::vec *>(rD + nr + u) = typename R::vec{rb.v[0], rb.v[1]};
}

// k_dic_update_forward_rb (kUpdate) or k_dic_forward_rb with two red-black
// pairs per lane (the lanes and partial sums of k_amul_dot_rb2): the black
// rows u, u + 1 take their red neighbours' rD, r (updated: r - alpha q) and
// mirrored slots as 16-byte loads one line or plane away, and their
// x-neighbours from the lane's red pair (slots -x and +x, which it loads) or
// the adjacent lane's; each row's recurrence is the pair kernel's term for
// term
template <bool kUpdate>
__global__ void __launch_bounds__(kCellBlock)
k_dic_forward_rb2(SolverParams sp, RBLayout L, const double *__restrict__ coef, const double *__restrict__ rD,
                  const double *__restrict__ q, double *__restrict__ r, double *__restrict__ w,
                  double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    const RBForm &f = L.f;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    const double alpha = kUpdate ? st->alpha : 0.0;
    const Rb2Lane l = rb2_lane(f);
    const int64_t u = l.u, pos = l.pos;
    const int32_t par = l.par;
    const R z = lanes_zero<double, 2>();
    // the red r a black row uses: updated (the value the update kernel would
    // store), or as it is
    auto upd = [&](double rv, double qv) { return kUpdate ? rv - alpha * qv : rv; };
    // the lane's red pair: rD, r, slots -x and +x
    R rdr = z, rrr = z, s2 = z, s3 = z;
    if (l.tv) {
        rdr = lanes_load<double, 2>(rD, u);
        const R r0 = lanes_load<double, 2>(r, u), q0 = kUpdate ? lanes_load<double, 2>(q, u) : z;
#pragma unroll
        for (int k = 0; k < 2; ++k) rrr.v[k] = upd(r0.v[k], q0.v[k]);
        s2 = lanes_load<double, 2>(coef, 2 * nr + u);
        s3 = lanes_load<double, 2>(coef, 3 * nr + u);
    }
    double rd_m1 = lane_from_below(rdr.v[1]), rr_m1 = lane_from_below(rrr.v[1]), s3_m1 = lane_from_below(s3.v[1]);
    double rd_p2 = lane_from_above(rdr.v[0]), rr_p2 = lane_from_above(rrr.v[0]), s2_p2 = lane_from_above(s2.v[0]);
    double acc[1] = {0.0};
    if (l.tv) {
        if (!l.below_ok && pos >= 2) {
            rd_m1 = rD[u - 1];
            rr_m1 = upd(r[u - 1], kUpdate ? q[u - 1] : 0.0);
            s3_m1 = coef[3 * nr + u - 1];
        }
        if (!l.above_ok && pos + 2 <= h - 1) {
            rd_p2 = rD[u + 2];
            rr_p2 = upd(r[u + 2], kUpdate ? q[u + 2] : 0.0);
            s2_p2 = coef[2 * nr + u + 2];
        }
        // red neighbours one plane down (slot +z), one line down (+y), one line
        // up (-y), one plane up (-z): rD, updated r, the mirrored slot
        const int64_t off[4] = {-H, -h, h, H};
        const int slot[4] = {5, 4, 1, 0};
        const bool has[4] = {l.zlo, l.ylo, l.yhi, l.zhi};
        R nrd[4], nrr[4], nsl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            nrd[i] = nrr[i] = nsl[i] = z;
            if (has[i]) {
                const int64_t v = u + off[i];
                nrd[i] = lanes_load<double, 2>(rD, v);
                const R r0 = lanes_load<double, 2>(r, v), q0 = kUpdate ? lanes_load<double, 2>(q, v) : z;
#pragma unroll
                for (int k = 0; k < 2; ++k) nrr[i].v[k] = upd(r0.v[k], q0.v[k]);
                nsl[i] = lanes_load<double, 2>(coef, slot[i] * nr + v);
            }
        }
        const R rb = lanes_load<double, 2>(r, nr + u), qb = kUpdate ? lanes_load<double, 2, true>(q, nr + u) : z;
        const R rdb = lanes_load<double, 2>(rD, nr + u);
        R rc, wv;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t pk = pos + k;
            const double c = upd(rb.v[k], qb.v[k]);
            rc.v[k] = c;
            if (kUpdate) acc[0] += fabs(c);
            const double rd = rdb.v[k];
            double wc = rd * c;
            // x entries: the red cells at u + k - par (slot +x) and u + k + 1 - par (slot -x)
            const double a2 = par ? (k == 0 ? s3_m1 : s3.v[0]) : s3.v[k];
            const double d2 = par ? (k == 0 ? rd_m1 : rdr.v[0]) : rdr.v[k];
            const double o2 = par ? (k == 0 ? rr_m1 : rrr.v[0]) : rrr.v[k];
            const double a3 = par ? s2.v[k] : (k == 0 ? s2.v[1] : s2_p2);
            const double d3 = par ? rdr.v[k] : (k == 0 ? rdr.v[1] : rd_p2);
            const double o3 = par ? rrr.v[k] : (k == 0 ? rrr.v[1] : rr_p2);
            const bool ok[6] = {l.zlo, l.ylo, pk >= par, pk + 1 - par <= h - 1, l.yhi, l.zhi};
            const double a[6] = {nsl[0].v[k], nsl[1].v[k], a2, a3, nsl[2].v[k], nsl[3].v[k]};
            const double rdo[6] = {nrd[0].v[k], nrd[1].v[k], d2, d3, nrd[2].v[k], nrd[3].v[k]};
            const double ro[6] = {nrr[0].v[k], nrr[1].v[k], o2, o3, nrr[2].v[k], nrr[3].v[k]};
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (ok[j]) wc -= rd * a[j] * (rdo[j] * ro[j]);
            wv.v[k] = wc;
        }
        if (kUpdate) *reinterpret_cast<typename R::vec *>(r + nr + u) = typename R::vec{rc.v[0], rc.v[1]};
        *reinterpret_cast<typename R::vec *>(w + nr + u) = typename R::vec{wv.v[0], wv.v[1]};
    }
    if (kUpdate) {
        const int slots[1] = {kPartSumR};
        write_partials<1>(part, sp.grid, slots, acc);
    }
}

// k_dic_backward_rb_pair with two red-black pairs per lane: the red rows u,
// u + 1 (kUpdate: their update of r first), then the backward sweep from their
// black neighbours' w, with the w.r partials of the lane's red and black rows
// and (kUpdate) the red rows' |r| added to the forward kernel's partial of the
// same workgroup
template <bool kUpdate>
__global__ void __launch_bounds__(kCellBlock)
k_dic_backward_rb2(SolverParams sp, RBLayout L, const double *__restrict__ coef, const double *__restrict__ rD,
                   const double *__restrict__ q, double *__restrict__ r, double *__restrict__ w,
                   double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    const RBForm &f = L.f;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    const double alpha = kUpdate ? st->alpha : 0.0;
    const Rb2Lane l = rb2_lane(f);
    const int64_t u = l.u, pos = l.pos;
    const int32_t par = l.par;
    const R z = lanes_zero<double, 2>();
    const R wb = l.tv ? lanes_load<double, 2>(w, nr + u) : z;
    double wb_m1 = lane_from_below(wb.v[1]), wb_p2 = lane_from_above(wb.v[0]);
    double acc[2] = {0.0, 0.0};
    if (l.tv) {
        if (!l.below_ok && pos >= 2) wb_m1 = w[nr + u - 1];
        if (!l.above_ok && pos + 2 <= h - 1) wb_p2 = w[nr + u + 2];
        R sl[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) sl[j] = lanes_load<double, 2>(coef, j * nr + u);
        const int64_t off[4] = {-H, -h, h, H};
        const bool has[4] = {l.zlo, l.ylo, l.yhi, l.zhi};
        R nw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) nw[i] = has[i] ? lanes_load<double, 2>(w, nr + u + off[i]) : z;
        const R rdr = lanes_load<double, 2>(rD, u), rr = lanes_load<double, 2>(r, u);
        const R qr = kUpdate ? lanes_load<double, 2, true>(q, u) : z;
        const R rbk = lanes_load<double, 2>(r, nr + u);
        R rcv, wv;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t pk = pos + k;
            const double c = kUpdate ? rr.v[k] - alpha * qr.v[k] : rr.v[k];
            rcv.v[k] = c;
            if (kUpdate) acc[1] += fabs(c);
            const double rd = rdr.v[k];
            double wc = rd * c;
            // x entries: the black cells at u + k + par - 1 and u + k + par
            const double w2 = par ? wb.v[k] : (k == 0 ? wb_m1 : wb.v[0]);
            const double w3 = par ? (k == 0 ? wb.v[1] : wb_p2) : wb.v[k];
            const bool ok[6] = {l.zlo, l.ylo, pk + par - 1 >= 0, pk + par <= h - 1, l.yhi, l.zhi};
            const double wo[6] = {nw[0].v[k], nw[1].v[k], w2, w3, nw[2].v[k], nw[3].v[k]};
#pragma unroll
            for (int j = 5; j >= 0; --j)
                if (ok[j]) wc -= rd * sl[j].v[k] * wo[j];
            wv.v[k] = wc;
            acc[0] += wc * c + wb.v[k] * rbk.v[k];
        }
        if (kUpdate) *reinterpret_cast<typename R::vec *>(r + u) = typename R::vec{rcv.v[0], rcv.v[1]};
        *reinterpret_cast<typename R::vec *>(w + u) = typename R::vec{wv.v[0], wv.v[1]};
    }
    if (kUpdate) {
        const double black = part[kPartSumR * sp.grid + blockIdx.x];
        block_sum<kCellBlock, 2>(acc);
        if (threadIdx.x == 0) {
            part[kPartWr * sp.grid + blockIdx.x] = acc[0];
            part[kPartSumR * sp.grid + blockIdx.x] = black + acc[1];
        }
    } else {
        double a1[1] = {acc[0]};
        const int slots[1] = {kPartWr};
        write_partials<1>(part, sp.grid, slots, a1);
    }
}

// backward sweep on the red rows, one thread per half-index u (red row u),
// with the w.r partial sums of the red row and of the black row nr + u (its
// w from the forward sweep); sp.grid_amul workgroups (the slot's further
// partials hold the zeros the update wrote)
// kUpdate: after k_dic_update_forward_rb, the red row's r -= alpha q first,
// and the red rows' |r| added to the black rows' partial sums of the block
template <bool kUpdate>
__global__ void __launch_bounds__(kCellBlock)
k_dic_backward_rb_pair(SolverParams sp, RBLayout L, const double *__restrict__ coef,
                       const double *__restrict__ rD, const double *__restrict__ q, double *__restrict__ r,
                       double *__restrict__ w, double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t nr = L.f.nr;
    const int32_t u = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[2] = {0.0, 0.0};
    if (u < nr) {
        int64_t slot[6];
        int32_t col[6];
        bool ok[6];
        rb_row(L.f, u, slot, col, ok);
        double a[6], wo[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            a[j] = coef[slot[j]];
            wo[j] = w[col[j]];
        }
        const double rd = rD[u];
        double rc = r[u];
        if (kUpdate) {
            rc = rc - st->alpha * __builtin_nontemporal_load(&q[u]);
            r[u] = rc;
            acc[1] = fabs(rc);
        }
        double wc = rd * rc;
#pragma unroll
        for (int j = 5; j >= 0; --j)
            if (ok[j]) wc -= rd * a[j] * wo[j];
        w[u] = wc;
        acc[0] = wc * rc + w[nr + u] * r[nr + u];
    }
    if (kUpdate) {
        // the block's |r| partial: its black rows' (written by the forward
        // sweep, same workgroup index) plus its red rows'
        const double black = part[kPartSumR * sp.grid + blockIdx.x];
        block_sum<kCellBlock, 2>(acc);
        if (threadIdx.x == 0) {
            part[kPartWr * sp.grid + blockIdx.x] = acc[0];
            part[kPartSumR * sp.grid + blockIdx.x] = black + acc[1];
        }
    } else {
        double a1[1] = {acc[0]};
        const int slots[1] = {kPartWr};
        write_partials<1>(part, sp.grid, slots, a1);
    }
}

// face-order copy of the two-colour band coefficients: upper_f at its slot
__global__ void __launch_bounds__(kCellBlock)
k_rb_upper(int32_t F, RBForm rf, const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
           const double *__restrict__ coef, double *__restrict__ upper) {
    const int64_t f = static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x;
    if (f >= F) return;
    const int32_t u = owner[f];
    const int32_t d = rb_direction(rf, u, neighbour[f] - rf.nr);
    if (d >= 0) upper[f] = coef[static_cast<int64_t>(d) * rf.nr + u];
}

// ---------------------------------------------------------------------------
// One-workgroup reductions and the solver's scalar decisions (READING:
// OpenFOAM's PCG semantics):
//  kFinMean:  mean of x0; resets the state.
//  kFinStart: normFactor = sum(|wA - pA| + |b - pA|) + 1e-20, res0 = sum|r| /
//             normFactor; converged iff res0 < tol (the relative test cannot
//             pass at the start); the loop runs iff minIter > 0 or not
//             converged; first w.r.
//  kFinAlpha: p.Ap; singular iff |p.Ap| / normFactor < 1e-300 (ends the solve,
//             the iteration is not counted); alpha = wArA / p.Ap.
//  kFinBeta:  the iteration is counted; res = sum|r| / normFactor; the
//             convergence check is made while nIter < maxIter; the loop goes on
//             while (nIter < maxIter and not converged) or nIter < minIter;
//             beta = wArA_new / wArA.
// ---------------------------------------------------------------------------

template <int Mode>
__device__ __forceinline__ void finalize_state(const SolverParams &sp, const double *__restrict__ part,
                                               PcgState *__restrict__ st) {
    const int32_t G = sp.grid;
    if (Mode == kFinMean) {
        double v[1];
        const int slots[1] = {kPartSumX};
        reduce_partials<1>(part, G, slots, v);
        if (threadIdx.x == 0) {
            st->x_avg = v[0] / static_cast<double>(sp.n);
            st->n_iter = 0;
            st->done = 0;
            st->converged = 0;
            st->singular = 0;
            st->nonfinite = 0;
            st->alpha = 0.0;
            st->beta = 0.0;
            st->n_outer = 0;
            st->inner_iter = 0;
            st->inner_done = 0;
        }
    } else if (Mode == kFinStart) {
        double v[3];
        const int slots[3] = {kPartNf, kPartSumR, kPartWr};
        reduce_partials<3>(part, G, slots, v);
        if (threadIdx.x == 0) {
            const double nf = v[0] + 1e-20;
            const double res0 = v[1] / nf;
            const bool conv = check_conv(res0, res0, sp.tol, sp.rel_tol);
            const bool bad = !isfinite(res0) || !isfinite(v[2]);
            st->nf = nf;
            st->res0 = res0;
            st->res = res0;
            st->converged = conv ? 1 : 0;
            st->wArA = v[2];
            if (bad) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (!(sp.min_iter > 0 || !conv)) {
                st->done = 1;
            }
        }
    } else if (Mode == kFinAlpha) {
        if (st->done) return;
        // the Amul launch wrote sp.grid_amul partials
        double v[1];
        const int slots[1] = {kPartPq};
        reduce_partials<1>(part, G, sp.grid_amul, slots, v);
        if (threadIdx.x == 0) {
            const double pq = v[0];
            if (!isfinite(pq)) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (fabs(pq) / st->nf < 1e-300) {
                st->singular = 1;
                st->done = 1;
            } else {
                st->alpha = st->wArA / pq;
            }
        }
    } else if (Mode == kFinConv) {
        // the iteration's convergence decision from the update's |r| partials
        // alone (the multigrid cycle, which forms w, runs only if the solve
        // goes on)
        if (st->done) return;
        double v[1];
        const int slots[1] = {kPartSumR};
        reduce_partials<1>(part, G, sp.grid_upd, slots, v);
        if (threadIdx.x == 0) {
            const double res = v[0] / st->nf;
            const int32_t k = st->n_iter + 1;
            st->n_iter = k;
            const bool conv = (k < sp.max_iter) ? check_conv(res, st->res0, sp.tol, sp.rel_tol)
                                                : (st->converged != 0);
            const bool cont = (k < sp.max_iter && !conv) || k < sp.min_iter;
            st->res = res;
            st->converged = conv ? 1 : 0;
            if (!isfinite(res)) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (!cont) {
                st->done = 1;
            }
        }
    } else if (Mode == kFinBetaOnly) {
        if (st->done) return;
        double v[1];
        const int slots[1] = {kPartWr};
        reduce_partials<1>(part, G, sp.grid, slots, v);
        if (threadIdx.x == 0) {
            if (!isfinite(v[0])) {
                st->nonfinite = 1;
                st->done = 1;
            } else {
                st->beta = v[0] / st->wArA;
                st->wArA = v[0];
            }
        }
    } else {
        if (st->done) return;
        double v[2];
        const int slots[2] = {kPartSumR, kPartWr};
        reduce_partials<2>(part, G, sp.grid_upd, slots, v);       // the update's partials
        if (threadIdx.x == 0) {
            const double res = v[0] / st->nf;
            const int32_t k = st->n_iter + 1;
            st->n_iter = k;
            const bool conv = (k < sp.max_iter) ? check_conv(res, st->res0, sp.tol, sp.rel_tol)
                                                : (st->converged != 0);
            const bool cont = (k < sp.max_iter && !conv) || k < sp.min_iter;
            const bool bad = !isfinite(res) || !isfinite(v[1]);
            st->res = res;
            st->converged = conv ? 1 : 0;
            if (bad) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (!cont) {
                st->done = 1;
            } else {
                st->beta = v[1] / st->wArA;
                st->wArA = v[1];
            }
        }
    }
}

template <int Mode>
__global__ void __launch_bounds__(kFinBlock) k_finalize(SolverParams sp, const double *__restrict__ part,
                                                       PcgState *__restrict__ st) {
    finalize_state<Mode>(sp, part, st);
}

// ---------------------------------------------------------------------------
// The start of a step for several group members in one launch per kernel
// (the precision form's: x0 sums, mean, assembly fused with the start of the
// solve; then, after the FP32 scaling, the initial decision).  Member i takes
// workgroups gl.begin[i] .. (its own cell grid) or workgroup i (finalize).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCellBlock) k_grp_sum_x(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    sum_x_rows(b - gl.begin[i], m.sp, m.T, m.part);
}

template <int Mode>
__global__ void __launch_bounds__(kFinBlock) k_grp_fin(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const MemberDesc &m = tab[gl.slot[blockIdx.x]];
    finalize_state<Mode>(m.sp, m.part, m.st);
}

__global__ void __launch_bounds__(kCellBlock) k_grp_assemble(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    const int32_t blk = b - gl.begin[i];
    with_member_layout(m, [&](auto L) {
        assemble_rows<decltype(L), false, true, true>(blk, m.sp, m.rdt, m.DT, L, m.bface_start, m.bface_list,
                                                      m.bface_patch, m.bmag_sf, m.bdelta, m.patch_type,
                                                      m.patch_value, m.V, m.T, m.coef, nullptr, nullptr, nullptr,
                                                      m.diagB, m.srcB, nullptr, nullptr, m.diag_pc, m.r, m.rD,
                                                      m.part, m.st, m.sig32, m.r32, m.d32, m.p, nullptr, nullptr);
    });
}

void launch_group_setup(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(cells.begin[cells.n]));
    hipLaunchKernelGGL(k_grp_sum_x, grid, dim3(kCellBlock), 0, s, tab, cells);
    hipLaunchKernelGGL(k_grp_fin<kFinMean>, dim3(static_cast<unsigned>(cells.n)), dim3(kFinBlock), 0, s, tab, cells);
    hipLaunchKernelGGL(k_grp_assemble, grid, dim3(kCellBlock), 0, s, tab, cells);
}

void launch_group_fin_start(const MemberDesc *tab, const GroupLaunch &gl, hipStream_t s) {
    hipLaunchKernelGGL(k_grp_fin<kFinStart>, dim3(static_cast<unsigned>(gl.n)), dim3(kFinBlock), 0, s, tab, gl);
}

// Per-kernel timing only: keeps the GPU busy for `ticks` of its constant-rate
// wall clock so the host can enqueue the launches (and their event pairs) that
// follow before the GPU reaches them; the events then time the kernels rather
// than the host's launch rate.  Bounded by the clock, one thread.
__global__ void k_spin(int64_t ticks) {
    const int64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

__global__ void k_any_nonfinite(const double *__restrict__ a, int32_t n, PcgState *st) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(&st->flag, 1);
}

__global__ void k_clear_flag(PcgState *st) { st->flag = 0; }

// test hook: the solver state "not done", so that the preconditioner's kernels run
__global__ void k_clear_done(PcgState *st) { st->done = 0; }

// diagonal preconditioner as the solve applies it: w = (1/diag) r
__global__ void __launch_bounds__(kCellBlock)
k_diag_apply(int32_t n, const double *__restrict__ diagB, const double *__restrict__ r, double *__restrict__ w) {
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < n) {
        const double rd = 1.0 / diagB[c];
        w[c] = rd * r[c];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void carve_problem(Carver &cv, const lf_mesh *m, const lf_solver_opts &o, lf_problem *P) {
    const size_t N = m->N, F = m->F, B = m->B;
    const int32_t G = cell_blocks(m->N);
    auto *pt = cv.take<int32_t>(std::max<int32_t>(m->P, 1));
    auto *pv = cv.take<double>(std::max<int32_t>(m->P, 1));
    double *vec[11];
    for (auto &v : vec) v = cv.take<double>(N);
    auto *upper = cv.take<double>(F);
    auto *coef = cv.take<double>(coef_slots(m, use_bands(m, o), use_rb(m, o)));
    auto *ic = cv.take<double>(B);
    auto *bc = cv.take<double>(B);
    auto *tb = cv.take<double>(B);
    auto *part = cv.take<double>(static_cast<size_t>(kNumPart) * G);
    auto *state = cv.take<PcgState>(1);
    double *grad3 = nullptr, *lap_src = nullptr, *T_old = nullptr, *snb = nullptr;
    if (!m->orthogonal) {
        grad3 = cv.take<double>(3 * N);
        lap_src = cv.take<double>(N);
        T_old = cv.take<double>(N);
    }
    if (m->gface || m->gband) snb = cv.take<double>(B);
    // the Jacobi-scaled coefficients of diagonal FP64 solves on the block walk
    // (lf_problem_create decides; every problem that may take it has them)
    double *coefS = nullptr;
    if (o.precision == LF_PREC_FP64 && o.precond == LF_PC_DIAGONAL && use_bands(m, o) && m->n_bands == 3)
        coefS = cv.take<double>(3 * N);
    if (P) {
        P->coefS = coefS;
        P->grad3 = grad3; P->lap_src = lap_src; P->T_old = T_old; P->snb = snb;
        P->patch_type = pt; P->patch_value = pv;
        P->T = vec[0]; P->r = vec[1]; P->p = vec[2]; P->q = vec[3]; P->w = vec[4]; P->rD = vec[5];
        P->p2 = vec[6]; P->diag = vec[7]; P->source = vec[8]; P->diagB = vec[9]; P->srcB = vec[10];
        P->upper = upper; P->coef = coef; P->int_coeff = ic; P->bou_coeff = bc; P->Tb = tb; P->part = part;
        P->state = state;
    }
    if (o.precision == LF_PREC_MIXED) carve_mixed(cv, m, use_bands(m, o), P);
    if (o.precond == LF_PC_AMG) carve_amg(cv, m, P);
}

MeshRows mesh_rows(const lf_mesh *m) { return MeshRows{m->soff, m->scol, m->sface, m->rlen}; }

template <class Lay>
struct IsBandLayout : std::false_type {};
template <int K>
struct IsBandLayout<BandLayout<K>> : std::true_type {};

template <bool kFull, bool kSetup, bool kMixed>
static void launch_assemble_t(lf_problem *P, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    const double rdt = 1.0 / P->dt;
    const bool diag_pc = P->opts.precond == LF_PC_DIAGONAL;
    // band meshes: the correction's source is formed inside the assembly
    // (the gradient pass still runs first)
    const bool fused = P->nonorth && P->banded && !P->rb && m->gkband;
    // the set-up's form: 0 DIC or multigrid (r only), 1 diagonal (r, rD, p = w),
    // 2 diagonal on the Jacobi-scaled system (the scaled r, p and x into w)
    const bool js = kSetup && !kMixed && P->scaled;
    const int32_t pc_mode = diag_pc ? (js ? 2 : 1) : 0;
    double *xs = js ? P->w : nullptr;
    if (P->nonorth) launch_nonorth_source(P, s, !fused);
    with_layout(P, [&](auto lay) {
        using Lay = decltype(lay);
        const double *T_old = kSetup && P->nonorth && P->opts.n_nonorth_corr > 0 ? P->T_old : nullptr;
        if constexpr (IsBandLayout<Lay>::value) {
            if (fused) {
                auto kern = k_assemble<Lay, kFull, kSetup, kMixed, true>;
                LF_LAUNCH(P, LF_K_ASSEMBLE, s, kern, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, rdt, P->DT, lay,
                          m->rbface_start, m->rbface_list, m->bface_patch, m->bmag_sf, m->bdelta, P->patch_type,
                          P->patch_value, m->V, P->T, P->coef, P->upper, P->diag, P->source, P->diagB, P->srcB,
                          P->int_coeff, P->bou_coeff, pc_mode, P->r, P->rD, P->part, P->state, P->sig32,
                          P->r32, P->d32, P->p, nullptr, T_old, P->grad3, m->gkband, xs);
                return;
            }
        }
        if constexpr (std::is_same_v<Lay, RBLayout> && !kMixed) {
            if (P->rb2 && !P->nonorth && !diag_pc) {
                auto kern = k_assemble_rb2<kFull, kSetup>;
                LF_LAUNCH(P, LF_K_ASSEMBLE, s, kern, dim3(static_cast<unsigned>(P->sp.grid_upd)), dim3(kCellBlock),
                          0, s, P->sp, rdt, P->DT, lay, m->rbface_start, m->rbface_list, m->bface_patch, m->bmag_sf,
                          m->bdelta, P->patch_type, P->patch_value, m->V, P->T, P->coef, P->diag, P->source,
                          P->diagB, P->srcB, P->int_coeff, P->bou_coeff, P->r, P->part, P->state);
                return;
            }
        }
        auto kern = k_assemble<Lay, kFull, kSetup, kMixed>;
        LF_LAUNCH(P, LF_K_ASSEMBLE, s, kern, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, rdt, P->DT, lay,
                  m->rbface_start, m->rbface_list, m->bface_patch, m->bmag_sf, m->bdelta, P->patch_type,
                  P->patch_value, m->V, P->T, P->coef, P->upper, P->diag, P->source, P->diagB, P->srcB,
                  P->int_coeff, P->bou_coeff, pc_mode, P->r, P->rD, P->part, P->state, P->sig32,
                  P->r32, P->d32, P->p, P->nonorth ? P->lap_src : nullptr, T_old, nullptr, nullptr, xs);
    });
    if (kFull && P->rb && m->F > 0)
        hipLaunchKernelGGL(k_rb_upper, dim3(static_cast<unsigned>((m->F + kCellBlock - 1) / kCellBlock)),
                           dim3(kCellBlock), 0, s, m->F, rb_form(m), m->owner, m->neighbour, P->coef, P->upper);
    if (kFull && P->banded && m->F > 0) {
        BandOffsets bo{};
        bo.k = m->n_bands;
        for (int k = 0; k < m->n_bands; ++k) bo.d[k] = m->band_d[k];
        hipLaunchKernelGGL(k_band_upper, dim3(static_cast<unsigned>((m->F + kCellBlock - 1) / kCellBlock)),
                           dim3(kCellBlock), 0, s, m->F, m->N, bo, m->owner, m->neighbour, P->coef, P->upper);
    }
}

lf_status launch_assemble(lf_problem *P, bool full, hipStream_t s) {
    if (full) launch_assemble_t<true, false, false>(P, s);
    else launch_assemble_t<false, false, false>(P, s);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

template <int Mode>
void launch_fin(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_FINALIZE, s, k_finalize<Mode>, dim3(1), dim3(kFinBlock), 0, s, P->sp, P->part, P->state);
}

// mean of x0 = T, then the assembly fused with the start of the solve
lf_status launch_assemble_setup(lf_problem *P, hipStream_t s) {
    // the partial sums of T: written by the last solve's commit when nothing
    // has written T since, else taken here
    if (!P->sumx_valid) LF_LAUNCH(P, LF_K_SETUP1, s, k_sum_x, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->T, P->part);
    P->sumx_valid = false;
    launch_fin<kFinMean>(P, s);
    if (P->opts.precision == LF_PREC_MIXED) {
        launch_assemble_t<false, true, true>(P, s);
        launch_mx_scale(P, s);
        P->scaled32 = true;
    } else {
        launch_assemble_t<false, true, false>(P, s);
        if (P->scaled) {
            const lf_mesh *m = P->mesh;
            const unsigned g = static_cast<unsigned>((m->N / 2 + kCellBlock - 1) / kCellBlock);
            LF_LAUNCH(P, LF_K_SCALE, s, k_scale_coef, dim3(g), dim3(kCellBlock), 0, s, band_layout<3>(m), P->rD,
                      P->coef, P->coefS);
        }
    }
    LF_HIP(hipGetLastError());
    return LF_OK;
}

static void launch_direction(lf_problem *P, hipStream_t s) {
    if (P->scaled)          // p~ = r~ + beta p~, x~ += alpha p~ (x~ in w)
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction_scaled, dim3(static_cast<unsigned>(P->sp.grid_upd)),
                  dim3(kCellBlock), 0, s, P->sp, P->r, P->p, P->w, P->state);
    else if (P->opts.precond == LF_PC_DIAGONAL)
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction<true>, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->rD, P->r,
                  P->w, P->p, P->T, P->state);
    else
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction<false>, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->rD,
                  P->r, P->w, P->p, P->T, P->state);
}

template void launch_fin<kFinStart>(lf_problem *P, hipStream_t s);

// DIC sweeps w = M^-1 r (forward on the black rows, then backward on the red
// rows with the w.r partials of all rows)
static void launch_dic_sweeps(lf_problem *P, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    if (P->rb && P->rb2) {
        // the iteration kernels' two-pairs-per-lane form without the update
        // (its w.r partials fill the first sp.grid_upd entries; the assembly
        // wrote zeros in the others)
        const dim3 gb(static_cast<unsigned>(P->sp.grid_upd));
        LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward_rb2<false>, gb, dim3(kCellBlock), 0, s, P->sp, rb_layout(m),
                  P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
        LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward_rb2<false>, gb, dim3(kCellBlock), 0, s, P->sp,
                  rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
        return;
    }
    if (P->rb) {
        const int32_t nb = m->N - m->n_red;
        const dim3 gb(static_cast<unsigned>(std::max<int32_t>(1, (nb + kCellBlock - 1) / kCellBlock)));
        LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward_rb, gb, dim3(kCellBlock), 0, s, P->sp, rb_layout(m),
                  P->coef, P->rD, P->r, P->w, P->state);
        LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward_rb_pair<false>, gb, dim3(kCellBlock), 0, s, P->sp,
                  rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
        return;
    }
    LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, mesh_rows(m),
              P->coef, P->rD, P->r, P->w, P->state);
    LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward, cell_grid(P), dim3(kCellBlock), 0, s, P->sp,
              mesh_rows(m), P->coef, P->rD, P->r, P->w, P->part, P->state);
}

// after the fused assembly/setup kernel: preconditioner set-up (DIC), initial
// residual and convergence decision, first direction
static lf_status launch_setup(lf_problem *P, hipStream_t s) {
    const lf_mesh *m = P->mesh;
    const bool diag_pc = P->opts.precond == LF_PC_DIAGONAL;
    if (P->opts.precond == LF_PC_AMG) {
        launch_amg_galerkin(P, s);
        launch_amg_cycle(P, s);
    } else if (!diag_pc) {
        if (P->rb2)
            LF_LAUNCH(P, LF_K_DIC_RD, s, k_dic_rd_rb2, dim3(static_cast<unsigned>(P->sp.grid_upd)), dim3(kCellBlock),
                      0, s, rb_layout(m), P->diagB, P->coef, P->rD);
        else if (P->rb)
            LF_LAUNCH(P, LF_K_DIC_RD, s, k_dic_rd_rb, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, rb_layout(m),
                      P->diagB, P->coef, P->rD);
        else
            LF_LAUNCH(P, LF_K_DIC_RD, s, k_dic_rd, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, mesh_rows(m),
                      P->diagB, P->coef, P->rD);
        launch_dic_sweeps(P, s);
    }
    launch_fin<kFinStart>(P, s);
    // first direction p = w: with the diagonal preconditioner the assembly
    // kernel has written it already
    if (!diag_pc) launch_direction(P, s);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

// one PCG iteration after its direction update: q = A p, alpha, update of r,
// (DIC sweeps), convergence decision and beta, next direction (with the
// deferred x update)
static lf_status launch_iteration(lf_problem *P, hipStream_t s) {
    const bool diag_pc = P->opts.precond == LF_PC_DIAGONAL;
    with_layout(P, [&](auto lay) {
        if constexpr (std::is_same_v<decltype(lay), BandLayout<3>>) {
            if (P->scaled) {
                LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot_box_scaled, dim3(static_cast<unsigned>(P->bw.blocks)),
                          dim3(kBwBlock), 0, s, P->sp, lay, P->bw, P->coefS, P->p, P->q, P->part, P->state);
                return;
            }
            if (P->box) {
                LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot_box, dim3(static_cast<unsigned>(P->bw.blocks)),
                          dim3(kBwBlock), 0, s, P->sp, lay, P->bw, P->diagB, P->coef, P->p, P->q, P->part, P->state);
                return;
            }
        }
        constexpr int K = WalkBands<decltype(lay)>::value;
        if constexpr (K > 0) {
            if (P->walk) {
                LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot_walk<K>, dim3(static_cast<unsigned>(P->sp.grid_amul)),
                          dim3(kCellBlock), 0, s, P->sp, lay, P->diagB, P->coef, P->p, P->q, P->part, P->state);
                return;
            }
        }
        if constexpr (std::is_same_v<decltype(lay), RBLayout>) {
            if (P->rb2)
                LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot_rb2, dim3(static_cast<unsigned>(P->sp.grid_amul)),
                          dim3(kCellBlock), 0, s, P->sp, lay, P->diagB, P->coef, P->p, P->q, P->part, P->state);
            else
                LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot_rb, dim3(static_cast<unsigned>(P->sp.grid_amul)),
                          dim3(kCellBlock), 0, s, P->sp, lay, P->diagB, P->coef, P->p, P->q, P->part, P->state);
            return;
        }
        LF_LAUNCH(P, LF_K_AMUL_DOT, s, k_amul_dot<decltype(lay)>, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, lay,
                  P->diagB, P->coef, P->p, P->q, P->part, P->state);
    });
    if (P->fold) {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update_fold, dim3(static_cast<unsigned>(P->sp.grid_upd)), dim3(kCellBlock), 0,
                  s, P->sp, P->q, P->r, P->rD, P->part, P->state);
        LF_LAUNCH(P, LF_K_DIRECTION, s, k_direction_fold, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->rD, P->r,
                  P->p, P->T, P->part, P->state);
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    launch_fin<kFinAlpha>(P, s);
    if (P->rb && !diag_pc) {
        // red-black DIC on the two-colour band layout: the update of r fused
        // into the two sweeps
        const lf_mesh *m = P->mesh;
        const dim3 gb(static_cast<unsigned>(P->sp.grid_upd));
        if (P->rb2) {
            LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_forward_rb2<true>, gb, dim3(kCellBlock), 0, s, P->sp,
                      rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
            LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward_rb2<true>, gb, dim3(kCellBlock), 0, s, P->sp,
                      rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
        } else {
            LF_LAUNCH(P, LF_K_DIC_FORWARD, s, k_dic_update_forward_rb, gb, dim3(kCellBlock), 0, s, P->sp,
                      rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
            LF_LAUNCH(P, LF_K_DIC_BACKWARD, s, k_dic_backward_rb_pair<true>, gb, dim3(kCellBlock), 0, s, P->sp,
                      rb_layout(m), P->coef, P->rD, P->q, P->r, P->w, P->part, P->state);
        }
        launch_fin<kFinBeta>(P, s);
        launch_direction(P, s);
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    if (P->scaled) {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update_scaled, dim3(static_cast<unsigned>(P->sp.grid_upd)),
                  dim3(kCellBlock), 0, s, P->sp, P->q, P->r, P->rD, P->part, P->state);
    } else if (diag_pc) {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update<true>, dim3(static_cast<unsigned>(P->sp.grid_upd)),
                  dim3(kCellBlock), 0, s, P->sp, P->q, P->r,
                  P->rD, P->part, P->state);
    } else {
        LF_LAUNCH(P, LF_K_UPDATE, s, k_update<false>, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->q, P->r,
                  P->rD, P->part, P->state);
        if (P->opts.precond == LF_PC_AMG) {
            launch_fin<kFinConv>(P, s);
            launch_amg_cycle(P, s);
            launch_fin<kFinBetaOnly>(P, s);
            launch_direction(P, s);
            LF_HIP(hipGetLastError());
            return LF_OK;
        }
        launch_dic_sweeps(P, s);
    }
    launch_fin<kFinBeta>(P, s);
    launch_direction(P, s);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

void prof_lead(lf_problem *P, hipStream_t s) {
    if (!P->prof_on || s != P->stream) return;
    if (P->prof_ticks == 0) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, P->mesh->device) != hipSuccess ||
            khz <= 0)
            khz = 100000;
        P->prof_ticks = static_cast<int64_t>(khz) / 5;     // 200 us
    }
    hipLaunchKernelGGL(k_spin, dim3(1), dim3(1), 0, s, P->prof_ticks);
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

// graph of 2^lg iterations
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
    for (int lg = kMaxGraphLog; lg >= 0; --lg) {
        while (k >= (1 << lg)) {
            LF_TRY(get_iter_graph(P, lg));
            LF_HIP(hipGraphLaunch(P->g_iter[lg], s));
            k -= 1 << lg;
        }
    }
    return LF_OK;
}

// block of k iterations, then the state copy and ev[2]
static lf_status fp64_block(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    c.k = std::min<int32_t>(c.k, std::max<int32_t>(1, P->sp.max_iter + 1 - c.launched));
    prof_lead(P, s);
    LF_TRY(launch_iterations(P, c.k));
    c.launched += c.k;
    LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    LF_HIP(hipEventRecord(P->ev[2], s));
    return LF_OK;
}

lf_status fp64_start(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    prof_lead(P, s);
    LF_TRY(launch_setup(P, s));
    c.fixed_k = P->prof_on ? 1 : P->opts.iters_per_check;
    c.k = c.fixed_k > 0 ? c.fixed_k : std::max<int32_t>(1, P->last_iters > 0 ? P->last_iters + 1 : 8);
    c.launched = 0;
    c.stage = 0;
    return fp64_block(P, c);
}

lf_status fp64_advance(lf_problem *P, SolveCtx &c, bool *finished, lf_solve_stats *out) {
    hipStream_t s = P->stream;
    prof_flush(P);
    *finished = false;
    if (c.stage == 1) {
        const PcgState &h = *P->h_state;
        out->initial_residual = h.res0;
        out->final_residual = h.res;
        out->n_iter = h.n_iter;
        out->converged = h.converged;
        out->singular = h.singular;
        out->nonfinite = h.nonfinite;
        out->n_outer = 1;
        *finished = true;
        return LF_OK;
    }
    if (P->h_state->done) {
        prof_lead(P, s);
        if (P->scaled)
            LF_LAUNCH(P, LF_K_COMMIT, s, k_commit_scaled, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->T, P->w,
                      P->p, P->rD, P->part, P->state);
        else
            LF_LAUNCH(P, LF_K_COMMIT, s, k_commit, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->T, P->p,
                      P->part, P->state);
        LF_HIP(hipGetLastError());
        P->sumx_valid = true;
        LF_HIP(hipEventRecord(P->ev[2], s));
        c.stage = 1;
        return LF_OK;
    }
    if (c.launched > P->sp.max_iter + P->sp.min_iter + 8) {
        set_error("solver state never reached done after %d iterations", c.launched);
        return LF_ESTATE;
    }
    if (c.fixed_k <= 0) c.k = std::max<int32_t>(2, c.k / 2);
    return fp64_block(P, c);
}

// w = M r with the last assembled matrix (P->r to P->w, solver order): the
// preconditioner's set-up (DIC diagonal, multigrid coarse matrices) and one
// application
lf_status launch_precondition_hook(lf_problem *P) {
    const lf_mesh *m = P->mesh;
    hipStream_t s = P->stream;
    hipLaunchKernelGGL(k_clear_done, dim3(1), dim3(1), 0, s, P->state);
    if (P->opts.precond == LF_PC_DIAGONAL) {
        hipLaunchKernelGGL(k_diag_apply, cell_grid(P), dim3(kCellBlock), 0, s, m->N, P->diagB, P->r, P->w);
    } else if (P->opts.precond == LF_PC_AMG) {
        launch_amg_galerkin(P, s);
        launch_amg_cycle(P, s);
    } else {
        if (P->rb2)
            hipLaunchKernelGGL(k_dic_rd_rb2, dim3(static_cast<unsigned>(P->sp.grid_upd)), dim3(kCellBlock), 0, s,
                               rb_layout(m), P->diagB, P->coef, P->rD);
        else if (P->rb)
            hipLaunchKernelGGL(k_dic_rd_rb, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, rb_layout(m), P->diagB,
                               P->coef, P->rD);
        else
            hipLaunchKernelGGL(k_dic_rd, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, mesh_rows(m), P->diagB,
                               P->coef, P->rD);
        launch_dic_sweeps(P, s);
    }
    LF_HIP(hipGetLastError());
    return LF_OK;
}

lf_status launch_amul_hook(lf_problem *P, const double *x, double *y) {
    with_layout(P, [&](auto lay) {
        if constexpr (std::is_same_v<decltype(lay), RBLayout>) {
            if (P->rb2) {
                hipLaunchKernelGGL(k_amul_rb2, dim3(static_cast<unsigned>(P->sp.grid_amul)), dim3(kCellBlock), 0,
                                   P->stream, lay, P->diagB, P->coef, x, y);
                return;
            }
        }
        if constexpr (std::is_same_v<decltype(lay), BandLayout<3>>) {
            if (P->box) {
                hipLaunchKernelGGL(k_amul_box, dim3(static_cast<unsigned>(P->bw.blocks)), dim3(kBwBlock), 0,
                                   P->stream, lay, P->bw, P->diagB, P->coef, x, y);
                return;
            }
        }
        constexpr int K = WalkBands<decltype(lay)>::value;
        if constexpr (K > 0) {
            if (P->walk) {
                hipLaunchKernelGGL(k_amul_walk<K>, dim3(static_cast<unsigned>(P->sp.grid_amul)), dim3(kCellBlock), 0,
                                   P->stream, lay, P->diagB, P->coef, x, y);
                return;
            }
        }
        hipLaunchKernelGGL(k_amul<decltype(lay)>, cell_grid(P), dim3(kCellBlock), 0, P->stream, P->sp, lay,
                           P->diagB, P->coef, x, y);
    });
    LF_HIP(hipGetLastError());
    return LF_OK;
}

lf_status check_finite_device(lf_problem *P, const double *T, bool *ok) {
    const int32_t N = P->mesh->N;
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, P->stream, P->state);
    hipLaunchKernelGGL(k_any_nonfinite, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream, T, N,
                       P->state);
    LF_HIP(hipGetLastError());
    LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, P->stream));
    LF_HIP(hipStreamSynchronize(P->stream));
    *ok = P->h_state->flag == 0;
    return LF_OK;
}

}  // namespace lf
