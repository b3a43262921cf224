// Precision form: mixed-precision iterative refinement.
//
// The matrix is assembled in FP64.  Outer loop in FP64: r = b - A T (true
// residual, FP64 coefficients and T), res = sum|r| / normFactor with the
// normalisation factor of x0 = T_old, stop when res < tol.  Each pass solves
// A d = r approximately in FP32 vectors, coefficients and products, with FP64
// dot products, alpha and beta; then T += d in FP64.
//
// The inner system is the symmetrically scaled one: with s = sqrt(diag A),
// As = S^-1 A S^-1 has a unit diagonal, rs = r / s, and plain CG on
// As y = rs gives d = y / s.  In exact arithmetic its iterates are those of
// the diagonally preconditioned CG on A d = r (the same alpha, beta and
// w.r = rs.rs); in the loop it reads neither the diagonal nor its
// reciprocal.  s is sqrt(diag A) rounded to FP32 (the scaled diagonal is 1 to
// FP32 rounding); the FP32 coefficients a / (s_c s_n) are formed once per
// step from the FP64 ones.  The update y += alpha p of an iteration is applied by
// the next iteration's direction kernel (which reads p anyway), and the last
// one by the correction T += (y + alpha p) / s.
//
// A pass after the first continues the CG of the one before instead of
// restarting it (a reliable update in the sense of Sleijpen and van der Vorst,
// 1996, as used for mixed-precision CG by Clark et al., 2010): the FP64 true
// residual replaces the recurred one and the last search direction is kept,
// projected so that it is orthogonal to the new residual.  A restart would
// discard the Krylov space built so far; the option inner_restart keeps it.
//
// The inner solve of a pass stops when the L1 norm of the residual it sees,
// sum s_c |rs_c|, has fallen by inner_tol, or below half the outer target,
// whichever is larger.  The refinement runs until res < kTighten * tol
// (convergence is still reported against tol).  Every FP64 PCG that stops
// just below tol leaves an error of its own in T, against the exactly solved
// step (on the 256^3 graded box up to 2.6e-8 relative in the first step from
// a random field, a few 1e-9 on small meshes); stopping an order of magnitude
// lower keeps the precision form's own error a tenth of that (1.4e-9 there).
// Its distance to one particular FP64 solve stopped at tol is then that
// solve's error plus its own, and is not bounded by 1e-8 where the former
// exceeds it.
constexpr double kTighten = 0.1;
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>

#include "lf_solver.h"

namespace lf {

void carve_mixed(Carver &cv, const lf_mesh *m, bool banded, lf_problem *P) {
    const size_t N = m->N;
    auto *coef32 = cv.take<float>(coef_slots(m, banded));
    float *v32[7];
    for (auto &v : v32) v = cv.take<float>(N);
    if (P) {
        P->coef32 = coef32; P->diag32 = v32[0]; P->rD32 = v32[1]; P->r32 = v32[2];
        P->p32 = v32[3]; P->q32 = v32[4]; P->d32 = v32[5]; P->sig32 = v32[6];
    }
}

__device__ __forceinline__ bool inner_off(const PcgState *st) { return st->done || st->inner_done; }

// FP32 coefficients of the scaled matrix: a_cn / (s_c s_n), with s the FP32
// sqrt(diagB) that also scales the residual and the correction (the scaled
// diagonal is then 1 to FP32 rounding, and taken as 1).  Band layout: the face
// (c, c + d_k) at k n + c.
template <int K>
__device__ __forceinline__ void scale_row(const BandLayout<K> &L, int32_t c, double sc,
                                          const float *__restrict__ sig32, const double *__restrict__ coef,
                                          float *__restrict__ coef32) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t slot = static_cast<int64_t>(k) * L.n + c;
        const bool ok = c < L.n - L.d[k];      // otherwise no face: the slot holds 0
        const double sn = ok ? static_cast<double>(sig32[c + L.d[k]]) : 1.0;
        coef32[slot] = static_cast<float>(coef[slot] / (sc * sn));
    }
}

// Row layout: each coefficient is in both its rows; s_c s_n = s_n s_c, so the
// two copies stay equal and the scaled matrix symmetric.
__device__ __forceinline__ void scale_row(const SellLayout &L, int32_t c, double sc,
                                          const float *__restrict__ sig32, const double *__restrict__ coef,
                                          float *__restrict__ coef32) {
    int32_t idx = row_base(L.mr, c);
    const int32_t len = L.mr.rlen[c];
    for (int32_t j = 0; j < len; ++j, idx += kSlice)
        coef32[idx] = static_cast<float>(coef[idx] / (sc * static_cast<double>(sig32[L.mr.scol[idx]])));
}

// Two-colour band layout: a red row scales its six slots (the precision form
// does not take DIC, so this serves only to complete the layout set)
__device__ __forceinline__ void scale_row(const RBLayout &L, int32_t c, double sc,
                                          const float *__restrict__ sig32, const double *__restrict__ coef,
                                          float *__restrict__ coef32) {
    if (c >= L.f.nr) return;
    int64_t slot[6];
    int32_t col[6];
    bool ok[6];
    rb_row(L.f, c, slot, col, ok);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double sn = ok[j] ? static_cast<double>(sig32[col[j]]) : 1.0;
        coef32[slot[j]] = static_cast<float>(coef[slot[j]] / (sc * sn));
    }
}

template <class Lay>
__device__ __forceinline__ void mx_scale(int32_t blk, const SolverParams &sp, const Lay &L,
                                         const float *__restrict__ sig32, const double *__restrict__ coef,
                                         float *__restrict__ coef32) {
    const int32_t c = blk * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) scale_row(L, c, static_cast<double>(sig32[c]), sig32, coef, coef32);
}

template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_scale(SolverParams sp, Lay L, const float *__restrict__ sig32, const double *__restrict__ coef,
           float *__restrict__ coef32) {
    mx_scale(static_cast<int32_t>(blockIdx.x), sp, L, sig32, coef, coef32);
}

// first inner iteration of a pass: p = rs, or, continuing the previous pass's
// CG, p = gamma rs + beta p; later: y += alpha p (the previous iteration's
// update), then p = rs + beta p; all FP32
// (workgroup blk of the problem's launch)
__device__ __forceinline__ void mx_direction(int32_t blk, const SolverParams &sp, const float *__restrict__ r32,
                                             float *__restrict__ p32, float *__restrict__ d32,
                                             const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    const bool first = st->inner_iter == 0;
    const bool cont = st->inner_cont != 0;
    const float beta = static_cast<float>(st->beta);
    const float alpha = static_cast<float>(st->alpha);
    const float gamma = static_cast<float>(st->gamma);
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row_at<kMxRows>(blk, j);
        if (c >= sp.n) continue;
        const float rc = r32[c];
        if (first) {
            p32[c] = cont ? gamma * rc + beta * p32[c] : rc;
        } else {
            const float pc = p32[c];
            // y is next needed an iteration later: stream it past the caches
            __builtin_nontemporal_store(__builtin_nontemporal_load(&d32[c]) + alpha * pc, &d32[c]);
            p32[c] = rc + beta * pc;
        }
    }
}

__global__ void __launch_bounds__(kCellBlock)
k_mx_direction(SolverParams sp, const float *__restrict__ r32, float *__restrict__ p32, float *__restrict__ d32,
               const PcgState *__restrict__ st) {
    mx_direction(static_cast<int32_t>(blockIdx.x), sp, r32, p32, d32, st);
}

// q = As p in FP32 (unit diagonal: p_c first, then the row's entries in
// order); FP64 partial sums of p.q
template <class Lay>
__device__ __forceinline__ void mx_amul_dot(int32_t blk, const SolverParams &sp, const Lay &L,
                                            const float *__restrict__ coef32, const float *__restrict__ p32,
                                            float *__restrict__ q32, double *__restrict__ part,
                                            const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    double acc[1] = {0.0};
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row_at<kMxRows>(blk, j);
        if (c >= sp.n) continue;
        const float pc = p32[c];
        const float qc = layout_dot(L, c, coef32, p32, pc);
        __builtin_nontemporal_store(qc, &q32[c]);
        acc[0] += static_cast<double>(qc) * static_cast<double>(pc);
    }
    const int slots[1] = {kPartPq};
    write_partials_at<1>(part, sp.grid_mx, blk, slots, acc);
}

template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_amul_dot(SolverParams sp, Lay L, const float *__restrict__ coef32, const float *__restrict__ p32,
              float *__restrict__ q32, double *__restrict__ part, const PcgState *__restrict__ st) {
    mx_amul_dot(static_cast<int32_t>(blockIdx.x), sp, L, coef32, p32, q32, part, st);
}

// the same product by the row walk (band layouts with two or more bands):
// sp.grid_mx_amul workgroups, whose partials fill the start of the p.q slot
// (slots sp.grid_mx apart)
template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_mx_amul_dot_walk(SolverParams sp, BandLayout<K> L, const float *__restrict__ coef32,
                   const float *__restrict__ p32, float *__restrict__ q32, double *__restrict__ part,
                   const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    double acc[1] = {band_walk<K, true, true, float>(L, nullptr, coef32, p32, q32)};
    const int slots[1] = {kPartPq};
    write_partials<1>(part, sp.grid_mx, slots, acc);
}

// the same product by the block walk of a box, four rows per lane (bw.blocks
// workgroups of kBwBlock threads, whose partials fill the start of the p.q slot)
__global__ void __launch_bounds__(kBwBlock)
k_mx_amul_dot_box(SolverParams sp, BandLayout<3> L, BoxWalk bw, const float *__restrict__ coef32,
                  const float *__restrict__ p32, float *__restrict__ q32, double *__restrict__ part,
                  const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    typedef Lanes<float, 4> R;
    double acc[1] = {0.0};
    box_walk<float, 4, false, true>(L, bw, nullptr, coef32, p32, [&](int64_t c, const R &qc, const R &pc, const R &) {
        lanes_store_stream(q32, c, qc);
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[0] += static_cast<double>(qc.v[w]) * static_cast<double>(pc.v[w]);
    });
    const int slots[1] = {kPartPq};
    write_partials<1, kBwBlock>(part, sp.grid_mx, slots, acc);
}

// rs -= alpha q (FP32); FP64 partials of the L1 norm s|rs| and of rs.rs
__device__ __forceinline__ void mx_update(int32_t blk, const SolverParams &sp, const float *__restrict__ q32,
                                          const float *__restrict__ sig32, float *__restrict__ r32,
                                          double *__restrict__ part, const PcgState *__restrict__ st) {
    if (inner_off(st)) return;
    const float alpha = static_cast<float>(st->alpha);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kMxRows; ++j) {
        const int32_t c = cell_row_at<kMxRows>(blk, j);
        if (c >= sp.n) continue;
        const float rc = r32[c] - alpha * __builtin_nontemporal_load(&q32[c]);
        r32[c] = rc;
        acc[0] += fabs(static_cast<double>(sig32[c]) * static_cast<double>(rc));
        acc[1] += static_cast<double>(rc) * static_cast<double>(rc);
    }
    const int slots[2] = {kPartSumR, kPartWr};
    write_partials_at<2>(part, sp.grid_mx, blk, slots, acc);
}

__global__ void __launch_bounds__(kCellBlock)
k_mx_update(SolverParams sp, const float *__restrict__ q32, const float *__restrict__ sig32,
            float *__restrict__ r32, double *__restrict__ part, const PcgState *__restrict__ st) {
    mx_update(static_cast<int32_t>(blockIdx.x), sp, q32, sig32, r32, part, st);
}

// T += d = (y + alpha p) / s in FP64, alpha p being the last inner update
// when it is still pending
__device__ __forceinline__ void mx_correct(int32_t blk, const SolverParams &sp, double *__restrict__ T,
                                           const float *__restrict__ d32, const float *__restrict__ p32,
                                           const float *__restrict__ sig32, const PcgState *__restrict__ st) {
    if (st->done) return;
    const bool pend = st->inner_pend != 0;
    const float alpha = static_cast<float>(st->alpha);
    const int32_t c = blk * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) {
        float y = d32[c];
        if (pend) y += alpha * p32[c];
        T[c] += static_cast<double>(y) / static_cast<double>(sig32[c]);
    }
}

__global__ void __launch_bounds__(kCellBlock)
k_mx_correct(SolverParams sp, double *__restrict__ T, const float *__restrict__ d32, const float *__restrict__ p32,
             const float *__restrict__ sig32, const PcgState *__restrict__ st) {
    mx_correct(static_cast<int32_t>(blockIdx.x), sp, T, d32, p32, sig32, st);
}

// one row of a pass end: from ax = (A T)_c, the FP64 residual r and the start
// of the next pass, which runs if the outer check does not stop the solve:
// rs = r / s rounded to FP32, y = 0; partial sums of |r|, s|rs|, rs.rs and,
// when the pass that just ended has a direction p (it iterated), rs.p
__device__ __forceinline__ void pass_end_row(int64_t c, double ax, double db, bool keep,
                                             const double *__restrict__ srcB, const float *__restrict__ p32,
                                             float *__restrict__ r32, float *__restrict__ d32, double (&acc)[4]) {
    const double rc = srcB[c] - ax;
    acc[0] += fabs(rc);
    const double sg = static_cast<float>(sqrt(db));     // the s of the scaled system
    const float rs = static_cast<float>(rc / sg);
    r32[c] = rs;
    d32[c] = 0.0f;
    acc[1] += fabs(sg * static_cast<double>(rs));
    acc[2] += static_cast<double>(rs) * static_cast<double>(rs);
    if (keep) acc[3] += static_cast<double>(rs) * static_cast<double>(p32[c]);
}

// true residual r = b - A T in FP64 and the start of the next pass (above)
template <class Lay>
__device__ __forceinline__ void mx_residual(int32_t blk, const SolverParams &sp, const Lay &L,
                                            const double *__restrict__ diagB, const double *__restrict__ coef,
                                            const double *__restrict__ srcB, const double *__restrict__ T,
                                            const float *__restrict__ p32, float *__restrict__ r32,
                                            float *__restrict__ d32, double *__restrict__ part,
                                            const PcgState *__restrict__ st) {
    if (st->done) return;
    const bool keep = st->inner_iter > 0;
    const int32_t c = blk * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < sp.n) {
        const double db = diagB[c];
        pass_end_row(c, layout_dot(L, c, coef, T, db * T[c]), db, keep, srcB, p32, r32, d32, acc);
    }
    const int slots[4] = {kPartSumR, kPartSumR32, kPartWr32, kPartRp32};
    write_partials_at<4>(part, sp.grid, blk, slots, acc);
}

template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_residual(SolverParams sp, Lay L, const double *__restrict__ diagB, const double *__restrict__ coef,
              const double *__restrict__ srcB, const double *__restrict__ T, const float *__restrict__ p32,
              float *__restrict__ r32, float *__restrict__ d32, double *__restrict__ part,
              const PcgState *__restrict__ st) {
    mx_residual(static_cast<int32_t>(blockIdx.x), sp, L, diagB, coef, srcB, T, p32, r32, d32, part, st);
}

// the same residual by the row walk (sp.grid_amul workgroups)
template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_mx_residual_walk(SolverParams sp, BandLayout<K> L, const double *__restrict__ diagB,
                   const double *__restrict__ coef, const double *__restrict__ srcB, const double *__restrict__ T,
                   const float *__restrict__ p32, float *__restrict__ r32, float *__restrict__ d32,
                   double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const bool keep = st->inner_iter > 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    band_walk_rows<K, true, false>(L, diagB, coef, T, [&](int64_t c, double ax, double, double db) {
        pass_end_row(c, ax, db, keep, srcB, p32, r32, d32, acc);
    });
    const int slots[4] = {kPartSumR, kPartSumR32, kPartWr32, kPartRp32};
    write_partials<4>(part, sp.grid, slots, acc);
}

// the same residual by the block walk of a box (bw.blocks workgroups)
__global__ void __launch_bounds__(kBwBlock)
k_mx_residual_box(SolverParams sp, BandLayout<3> L, BoxWalk bw, const double *__restrict__ diagB,
                  const double *__restrict__ coef, const double *__restrict__ srcB, const double *__restrict__ T,
                  const float *__restrict__ p32, float *__restrict__ r32, float *__restrict__ d32,
                  double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const bool keep = st->inner_iter > 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    typedef Lanes<double, 2> R;
    typedef float F2 __attribute__((ext_vector_type(2)));
    box_walk<double, 2, true, false>(L, bw, diagB, coef, T, [&](int64_t c, const R &ax, const R &, const R &db) {
        // the two rows as pass_end_row takes them, with 16- and 8-byte accesses
        const R b = lanes_load<double, 2>(srcB, c);
        const F2 pp = keep ? *reinterpret_cast<const F2 *>(p32 + c) : F2{0.0f, 0.0f};
        F2 rs2;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const double rc = b.v[w] - ax.v[w];
            acc[0] += fabs(rc);
            const double sg = static_cast<float>(sqrt(db.v[w]));
            const float rs = static_cast<float>(rc / sg);
            rs2[w] = rs;
            acc[1] += fabs(sg * static_cast<double>(rs));
            acc[2] += static_cast<double>(rs) * static_cast<double>(rs);
            if (keep) acc[3] += static_cast<double>(rs) * static_cast<double>(pp[w]);
        }
        *reinterpret_cast<F2 *>(r32 + c) = rs2;
        *reinterpret_cast<F2 *>(d32 + c) = F2{0.0f, 0.0f};
    });
    const int slots[4] = {kPartSumR, kPartSumR32, kPartWr32, kPartRp32};
    write_partials<4, kBwBlock>(part, sp.grid, slots, acc);
}

// one-workgroup decisions of the refinement
enum MxFin : int { kMxInnerStart = 0, kMxAlpha = 1, kMxBeta = 2, kMxOuter = 3 };

template <int Mode>
__device__ __forceinline__ void mx_finalize(const SolverParams &sp, const double *__restrict__ part,
                                            PcgState *__restrict__ st) {
    // partials per slot: the FP32 inner kernels use their own grid
    const int32_t G = (Mode == kMxAlpha || Mode == kMxBeta) ? sp.grid_mx : sp.grid;
    if (Mode == kMxInnerStart) {
        if (st->done) return;
        // the first pass starts from the assembly's partials (sp.grid of them),
        // later ones from the residual launch's (sp.grid_amul)
        double v[3];
        const int slots[3] = {kPartSumR32, kPartWr32, kPartRp32};
        reduce_partials<3>(part, G, st->n_outer == 0 ? sp.grid : sp.grid_amul, slots, v);
        if (threadIdx.x == 0) {
            const double target = fmax(sp.inner_tol * v[0], 0.5 * kTighten * sp.tol * st->nf);
            // a later pass continues the CG of the one before (which iterated):
            // the true residual replaces the recurred one, and the last
            // direction p is kept, made orthogonal to it (rs.p = 0, which CG's
            // alpha = rs.rs / p.Ap assumes): p = gamma rs + beta p with
            // beta = rs.rs / (rs.rs before the replacement) and
            // gamma = 1 - beta rs.p / rs.rs
            const bool cont = !sp.inner_restart && st->n_outer > 0 && st->inner_iter > 0 && st->wArA > 0.0 &&
                              v[1] > 0.0 && isfinite(v[1]) && isfinite(v[2]);
            st->inner_cont = cont ? 1 : 0;
            if (cont) {
                const double beta = v[1] / st->wArA;
                st->beta = beta;
                st->gamma = 1.0 - beta * (v[2] / v[1]);
            }
            st->inner_target = target;
            st->inner_iter = 0;
            st->inner_pend = 0;
            st->alpha = 0.0;
            st->wArA = v[1];
            st->inner_done = (v[0] <= target || !(v[1] > 0.0)) ? 1 : 0;
            if (!isfinite(v[0]) || !isfinite(v[1])) {
                st->nonfinite = 1;
                st->done = 1;
            }
        }
    } else if (Mode == kMxAlpha) {
        if (inner_off(st)) return;
        // the Amul launch wrote sp.grid_mx_amul partials
        double v[1];
        const int slots[1] = {kPartPq};
        reduce_partials<1>(part, G, sp.grid_mx_amul, slots, v);
        if (threadIdx.x == 0) {
            const double pq = v[0];
            st->inner_pend = 0;              // the direction kernel applied the previous update
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
            st->inner_pend = 1;              // y += alpha p of this iteration is pending
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
        reduce_partials<1>(part, G, sp.grid_amul, slots, v);     // the residual launch's partials
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
__global__ void __launch_bounds__(kFinBlock) k_mx_finalize(SolverParams sp, const double *__restrict__ part,
                                                          PcgState *__restrict__ st) {
    mx_finalize<Mode>(sp, part, st);
}

// ---------------------------------------------------------------------------
// The inner iteration of several problems in one launch per kernel (a group:
// lf_group_*).  Member i of a launch takes its workgroups gl.begin[i] ..
// gl.begin[i+1] - 1, which run the same rows and write the same partials as
// workgroups 0 .. of its own launch; the finalize launches take one workgroup
// per member.  Each problem's arithmetic and sums are therefore those of its
// own launches, whatever else shares the launch.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCellBlock)
k_grp_direction(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    mx_direction(b - gl.begin[i], m.sp, m.r32, m.p32, m.d32, m.st);
}

__global__ void __launch_bounds__(kCellBlock)
k_grp_amul_dot(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    const int32_t blk = b - gl.begin[i];
    with_member_layout(m, [&](auto L) { mx_amul_dot(blk, m.sp, L, m.coef32, m.p32, m.q32, m.part, m.st); });
}

__global__ void __launch_bounds__(kCellBlock)
k_grp_update(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    mx_update(b - gl.begin[i], m.sp, m.q32, m.sig32, m.r32, m.part, m.st);
}

template <int Mode>
__global__ void __launch_bounds__(kFinBlock) k_grp_finalize(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const MemberDesc &m = tab[gl.slot[blockIdx.x]];
    mx_finalize<Mode>(m.sp, m.part, m.st);
}

// every member's solver state into out[slot]
__global__ void k_grp_gather(const MemberDesc *__restrict__ tab, GroupLaunch gl, PcgState *__restrict__ out) {
    const int32_t i = static_cast<int32_t>(blockIdx.x);
    const int32_t n = static_cast<int32_t>(sizeof(PcgState) / sizeof(int32_t));
    const int32_t *src = reinterpret_cast<const int32_t *>(tab[gl.slot[i]].st);
    int32_t *dst = reinterpret_cast<int32_t *>(out + gl.slot[i]);
    for (int32_t t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

// the refinement's outer work of the launch's members (cell grids: gl.begin
// from each member's sp.grid; finalize: one workgroup per member)
__global__ void __launch_bounds__(kCellBlock)
k_grp_scale(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    const int32_t blk = b - gl.begin[i];
    with_member_layout(m, [&](auto L) { mx_scale(blk, m.sp, L, m.sig32, m.coef, m.coef32w); });
}

__global__ void __launch_bounds__(kCellBlock)
k_grp_correct(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    mx_correct(b - gl.begin[i], m.sp, m.T, m.d32, m.p32, m.sig32, m.st);
}

__global__ void __launch_bounds__(kCellBlock)
k_grp_residual(const MemberDesc *__restrict__ tab, GroupLaunch gl) {
    const int32_t b = static_cast<int32_t>(blockIdx.x), i = group_member(gl, b);
    const MemberDesc &m = tab[gl.slot[i]];
    const int32_t blk = b - gl.begin[i];
    with_member_layout(m, [&](auto L) {
        mx_residual(blk, m.sp, L, m.diagB, m.coef, m.srcB, m.T, m.p32, m.r32, m.d32, m.part, m.st);
    });
}

void launch_group_scale(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s) {
    hipLaunchKernelGGL(k_grp_scale, dim3(static_cast<unsigned>(cells.begin[cells.n])), dim3(kCellBlock), 0, s, tab,
                       cells);
}

void launch_group_pass_start(const MemberDesc *tab, const GroupLaunch &gl, hipStream_t s) {
    hipLaunchKernelGGL(k_grp_finalize<kMxInnerStart>, dim3(static_cast<unsigned>(gl.n)), dim3(kFinBlock), 0, s,
                       tab, gl);
}

// the end of a refinement pass: correction, FP64 residual, outer check
void launch_group_pass_end(const MemberDesc *tab, const GroupLaunch &cells, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(cells.begin[cells.n]));
    hipLaunchKernelGGL(k_grp_correct, grid, dim3(kCellBlock), 0, s, tab, cells);
    hipLaunchKernelGGL(k_grp_residual, grid, dim3(kCellBlock), 0, s, tab, cells);
    hipLaunchKernelGGL(k_grp_finalize<kMxOuter>, dim3(static_cast<unsigned>(cells.n)), dim3(kFinBlock), 0, s, tab,
                       cells);
}

// one inner iteration of the launch's members (grid sizes from gl)
void launch_group_iteration(const MemberDesc *tab, const GroupLaunch &gl, hipStream_t s) {
    const dim3 blk(kCellBlock), fin(kFinBlock), cells(static_cast<unsigned>(gl.begin[gl.n])),
        each(static_cast<unsigned>(gl.n));
    hipLaunchKernelGGL(k_grp_direction, cells, blk, 0, s, tab, gl);
    hipLaunchKernelGGL(k_grp_amul_dot, cells, blk, 0, s, tab, gl);
    hipLaunchKernelGGL(k_grp_finalize<kMxAlpha>, each, fin, 0, s, tab, gl);
    hipLaunchKernelGGL(k_grp_update, cells, blk, 0, s, tab, gl);
    hipLaunchKernelGGL(k_grp_finalize<kMxBeta>, each, fin, 0, s, tab, gl);
}

void launch_group_gather(const MemberDesc *tab, const GroupLaunch &gl, PcgState *out, hipStream_t s) {
    hipLaunchKernelGGL(k_grp_gather, dim3(static_cast<unsigned>(gl.n)), dim3(64), 0, s, tab, gl, out);
}

// the descriptor of a problem in a group
MemberDesc member_desc(const lf_problem *P) {
    MemberDesc m{};
    const lf_mesh *msh = P->mesh;
    m.sp = P->sp;
    m.kind = P->banded ? msh->n_bands : 0;
    m.n = msh->N;
    for (int k = 0; k < 4; ++k) m.d[k] = k < msh->n_bands ? msh->band_d[k] : 0;
    m.diag_pc = P->opts.precond == LF_PC_DIAGONAL ? 1 : 0;
    m.rdt = 1.0 / P->dt;
    m.DT = P->DT;
    m.mr = mesh_rows(msh);
    if (P->banded) {
        m.mag_sf = msh->band_mag_sf;
        m.delta = msh->band_delta;
    } else {
        m.mag_sf = msh->mag_sf;
        m.delta = msh->delta;
        m.emag_sf = msh->emag_sf;
        m.edelta = msh->edelta;
    }
    m.bface_start = msh->rbface_start;
    m.bface_list = msh->rbface_list;
    m.bface_patch = msh->bface_patch;
    m.bmag_sf = msh->bmag_sf;
    m.bdelta = msh->bdelta;
    m.V = msh->V;
    m.patch_type = P->patch_type;
    m.patch_value = P->patch_value;
    m.iperm = msh->iperm;
    m.T = P->T;
    m.coef = P->coef;
    m.diagB = P->diagB;
    m.srcB = P->srcB;
    m.r = P->r;
    m.rD = P->rD;
    m.p = P->p;
    m.coef32 = P->coef32;
    m.coef32w = P->coef32;
    m.sig32 = P->sig32;
    m.r32 = P->r32;
    m.p32 = P->p32;
    m.d32 = P->d32;
    m.q32 = P->q32;
    m.part = P->part;
    m.st = P->state;
    return m;
}

template <int Mode>
static void launch_mx_fin(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_FINALIZE, s, k_mx_finalize<Mode>, dim3(1), dim3(kFinBlock), 0, s, P->sp, P->part, P->state);
}

static void launch_inner_iteration(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_INNER_DIRECTION, s, k_mx_direction, mx_grid(P), dim3(kCellBlock), 0, s, P->sp, P->r32,
              P->p32, P->d32, P->state);
    with_layout(P, [&](auto lay) {
        if constexpr (std::is_same_v<decltype(lay), BandLayout<3>>) {
            if (P->box32) {
                LF_LAUNCH(P, LF_K_INNER_AMUL_DOT, s, k_mx_amul_dot_box, dim3(static_cast<unsigned>(P->bw32.blocks)),
                          dim3(kBwBlock), 0, s, P->sp, lay, P->bw32, P->coef32, P->p32, P->q32, P->part, P->state);
                return;
            }
        }
        constexpr int K = WalkBands<decltype(lay)>::value;
        if constexpr (K > 0) {
            if (P->walk) {
                LF_LAUNCH(P, LF_K_INNER_AMUL_DOT, s, k_mx_amul_dot_walk<K>,
                          dim3(static_cast<unsigned>(P->sp.grid_mx_amul)), dim3(kCellBlock), 0, s, P->sp, lay,
                          P->coef32, P->p32, P->q32, P->part, P->state);
                return;
            }
        }
        LF_LAUNCH(P, LF_K_INNER_AMUL_DOT, s, k_mx_amul_dot<decltype(lay)>, mx_grid(P), dim3(kCellBlock), 0, s,
                  P->sp, lay, P->coef32, P->p32, P->q32, P->part, P->state);
    });
    launch_mx_fin<kMxAlpha>(P, s);
    LF_LAUNCH(P, LF_K_INNER_UPDATE, s, k_mx_update, mx_grid(P), dim3(kCellBlock), 0, s, P->sp, P->q32, P->sig32,
              P->r32, P->part, P->state);
    launch_mx_fin<kMxBeta>(P, s);
}

// y = A32 x with the inner solve's FP32 coefficients (unit diagonal), in the
// form the inner solve uses (test hook)
template <class Lay>
__global__ void __launch_bounds__(kCellBlock)
k_mx_amul_hook(SolverParams sp, Lay L, const float *__restrict__ coef32, const float *__restrict__ x,
               float *__restrict__ y) {
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < sp.n) y[c] = layout_dot(L, c, coef32, x, x[c]);
}

template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_mx_amul_walk_hook(BandLayout<K> L, const float *__restrict__ coef32, const float *__restrict__ x,
                    float *__restrict__ y) {
    band_walk<K, false, true, float>(L, nullptr, coef32, x, y);
}

__global__ void __launch_bounds__(kBwBlock)
k_mx_amul_box_hook(BandLayout<3> L, BoxWalk bw, const float *__restrict__ coef32, const float *__restrict__ x,
                   float *__restrict__ y) {
    typedef Lanes<float, 4> R;
    box_walk<float, 4, false, true>(L, bw, nullptr, coef32, x, [&](int64_t c, const R &yc, const R &, const R &) {
#pragma unroll
        for (int w = 0; w < 4; ++w) y[c + w] = yc.v[w];
    });
}

lf_status launch_amul_inner_hook(lf_problem *P, const float *x, float *y) {
    with_layout(P, [&](auto lay) {
        if constexpr (std::is_same_v<decltype(lay), BandLayout<3>>) {
            if (P->box32) {
                hipLaunchKernelGGL(k_mx_amul_box_hook, dim3(static_cast<unsigned>(P->bw32.blocks)), dim3(kBwBlock), 0,
                                   P->stream, lay, P->bw32, P->coef32, x, y);
                return;
            }
        }
        constexpr int K = WalkBands<decltype(lay)>::value;
        if constexpr (K > 0) {
            if (P->walk) {
                hipLaunchKernelGGL(k_mx_amul_walk_hook<K>, dim3(static_cast<unsigned>(P->sp.grid_mx_amul)),
                                   dim3(kCellBlock), 0, P->stream, lay, P->coef32, x, y);
                return;
            }
        }
        hipLaunchKernelGGL(k_mx_amul_hook<decltype(lay)>, cell_grid(P), dim3(kCellBlock), 0, P->stream, P->sp, lay,
                           P->coef32, x, y);
    });
    LF_HIP(hipGetLastError());
    return LF_OK;
}

// k_mx_scale on a band layout whose first offset is 1 and whose other offsets
// and row count are even, two rows (c, c + 1, c even) per thread: 16-byte
// loads of the coefficients, 8-byte accesses of s and of the FP32 result;
// each value by scale_row's expression
template <int K>
__global__ void __launch_bounds__(kCellBlock)
k_mx_scale2(BandLayout<K> L, const float *__restrict__ sig32, const double *__restrict__ coef,
            float *__restrict__ coef32) {
    typedef float F2 __attribute__((ext_vector_type(2)));
    typedef double D2 __attribute__((ext_vector_type(2)));
    const int64_t n = L.n;
    const int64_t c = 2 * (static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x);
    if (c >= n) return;
    const F2 sv = *reinterpret_cast<const F2 *>(sig32 + c);
    const double sc[2] = {static_cast<double>(sv.x), static_cast<double>(sv.y)};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t d = L.d[k], slot = static_cast<int64_t>(k) * n + c;
        const D2 a = *reinterpret_cast<const D2 *>(coef + slot);
        double sn[2];
        if (k == 0) {
            // neighbours c + 1 (the pair's own) and c + 2
            sn[0] = static_cast<double>(sv.y);
            sn[1] = c + 1 < n - 1 ? static_cast<double>(sig32[c + 2]) : 1.0;
        } else if (c + 1 < n - d) {
            const F2 nv = *reinterpret_cast<const F2 *>(sig32 + c + d);
            sn[0] = static_cast<double>(nv.x);
            sn[1] = static_cast<double>(nv.y);
        } else {
            sn[0] = c < n - d ? static_cast<double>(sig32[c + d]) : 1.0;
            sn[1] = 1.0;
        }
        F2 o;
        o.x = static_cast<float>(a.x / (sc[0] * sn[0]));
        o.y = static_cast<float>(a.y / (sc[1] * sn[1]));
        *reinterpret_cast<F2 *>(coef32 + slot) = o;
    }
}

void launch_mx_scale(lf_problem *P, hipStream_t s) {
    with_layout(P, [&](auto lay) {
        using Lay = decltype(lay);
        constexpr int K = WalkBands<Lay>::value;
        if constexpr (K > 0) {
            bool pairs = lay.n % 2 == 0 && lay.d[0] == 1;
            for (int k = 1; k < K; ++k) pairs = pairs && lay.d[k] % 2 == 0;
            if (pairs) {
                const dim3 g(static_cast<unsigned>((lay.n / 2 + kCellBlock - 1) / kCellBlock));
                LF_LAUNCH(P, LF_K_MIXED_PREP, s, k_mx_scale2<K>, g, dim3(kCellBlock), 0, s, lay, P->sig32, P->coef,
                          P->coef32);
                return;
            }
        }
        LF_LAUNCH(P, LF_K_MIXED_PREP, s, k_mx_scale<Lay>, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, lay,
                  P->sig32, P->coef, P->coef32);
    });
}

// start of a refinement pass (rs, y = 0 and their partial sums were written
// by the kernel that formed the FP64 residual: the assembly or k_mx_residual)
static void launch_pass_start(lf_problem *P, hipStream_t s) { launch_mx_fin<kMxInnerStart>(P, s); }

// end of a pass: correction, true residual, outer decision
static void launch_pass_end(lf_problem *P, hipStream_t s) {
    LF_LAUNCH(P, LF_K_MIXED_CORRECT, s, k_mx_correct, cell_grid(P), dim3(kCellBlock), 0, s, P->sp, P->T, P->d32,
              P->p32, P->sig32, P->state);
    with_layout(P, [&](auto lay) {
        if constexpr (std::is_same_v<decltype(lay), BandLayout<3>>) {
            if (P->box) {
                LF_LAUNCH(P, LF_K_MIXED_RESIDUAL, s, k_mx_residual_box, dim3(static_cast<unsigned>(P->bw.blocks)),
                          dim3(kBwBlock), 0, s, P->sp, lay, P->bw, P->diagB, P->coef, P->srcB, P->T, P->p32, P->r32,
                          P->d32, P->part, P->state);
                return;
            }
        }
        constexpr int K = WalkBands<decltype(lay)>::value;
        if constexpr (K > 0) {
            if (P->walk) {
                LF_LAUNCH(P, LF_K_MIXED_RESIDUAL, s, k_mx_residual_walk<K>,
                          dim3(static_cast<unsigned>(P->sp.grid_amul)), dim3(kCellBlock), 0, s, P->sp, lay,
                          P->diagB, P->coef, P->srcB, P->T, P->p32, P->r32, P->d32, P->part, P->state);
                return;
            }
        }
        LF_LAUNCH(P, LF_K_MIXED_RESIDUAL, s, k_mx_residual<decltype(lay)>, cell_grid(P), dim3(kCellBlock), 0, s,
                  P->sp, lay, P->diagB, P->coef, P->srcB, P->T, P->p32, P->r32, P->d32, P->part, P->state);
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

// block of k inner iterations (k may be 0), then the state copy and ev[2]
static lf_status mixed_block(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    prof_lead(P, s);
    LF_TRY(launch_inner(P, c.k));
    c.launched += c.k;
    LF_HIP(hipMemcpyAsync(P->h_state, P->state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    LF_HIP(hipEventRecord(P->ev[2], s));
    return LF_OK;
}

// first block of refinement pass `pass`: as many iterations as that pass took
// in the last step (the counts repeat closely from step to step)
static int32_t predicted_inner(const lf_problem *P, int32_t pass) {
    const int32_t k = pass < lf_problem::kPassTrack ? P->last_inner[pass] : 0;
    return k > 0 ? k : 8;
}

lf_status mixed_start(lf_problem *P, SolveCtx &c) {
    hipStream_t s = P->stream;
    prof_lead(P, s);
    launch_fin<kFinStart>(P, s);      // normFactor, res0 and the initial decision (shared with FP64)
    launch_pass_start(P, s);
    LF_HIP(hipGetLastError());
    c.fixed_k = P->prof_on ? 1 : P->opts.iters_per_check;
    c.k = c.fixed_k > 0 ? c.fixed_k : predicted_inner(P, 0);
    c.launched = 0;
    c.stage = 0;
    return mixed_block(P, c);
}

// Host side of the refinement.  Iterations past the end of a pass (or of the
// solve) run as no-op launches, so the blocks are sized to what the pass is
// expected to need; after the pass that ended the last step the outer check
// is read back before another pass is enqueued (stage 1).
lf_status mixed_advance(lf_problem *P, SolveCtx &c, bool *finished, lf_solve_stats *out) {
    hipStream_t s = P->stream;
    prof_flush(P);
    *finished = false;
    const PcgState &h = *P->h_state;
    const bool adaptive = c.fixed_k <= 0;
    if (h.done) {
        out->initial_residual = h.res0;
        out->final_residual = h.res;
        out->n_iter = h.n_iter;
        out->converged = h.converged;
        out->singular = 0;
        out->nonfinite = h.nonfinite;
        out->n_outer = h.n_outer;
        P->last_outer = h.n_outer;
        *finished = true;
        return LF_OK;
    }
    if (c.launched > 4 * (P->sp.max_iter + 8) + 64 * P->sp.max_outer) {
        set_error("mixed solver never reached done after %d launched inner iterations", c.launched);
        return LF_ESTATE;
    }
    if (c.stage == 1) {
        // the outer check after a pass asked for another one
        c.stage = 0;
        prof_lead(P, s);
        launch_pass_start(P, s);
        LF_HIP(hipGetLastError());
        c.k = predicted_inner(P, h.n_outer);
        return mixed_block(P, c);
    }
    if (!h.inner_done) {
        // the pass needs more than predicted: small top-ups
        if (adaptive) c.k = 2;
        return mixed_block(P, c);
    }
    // pass finished: correct, check, and (unless it may have been the last one)
    // start the next pass, all no-ops once the solve is done
    const int32_t pass = h.n_outer;
    if (pass < lf_problem::kPassTrack) P->last_inner[pass] = h.inner_iter;
    prof_lead(P, s);
    launch_pass_end(P, s);
    LF_HIP(hipGetLastError());
    if (adaptive && P->last_outer > 0 && pass + 1 >= P->last_outer) {
        c.stage = 1;
        c.k = 0;
        return mixed_block(P, c);
    }
    launch_pass_start(P, s);
    LF_HIP(hipGetLastError());
    if (adaptive) c.k = predicted_inner(P, pass + 1);
    return mixed_block(P, c);
}

}  // namespace lf
