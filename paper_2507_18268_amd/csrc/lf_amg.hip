// Aggregation multigrid preconditioner (FP64) for meshes with the box form.
//
// The paper's conclusion names an algebraic multigrid library as the better
// alternative to the diagonal PCG.  Here the cycle is built on the box: level
// l + 1 aggregates the 2 x 2 x 2 blocks of level l (a side of odd length ends
// with a block one cell thick), every level is again a box numbered
// i + nx (j + ny k), so each level's matrix lives in the band layout and is
// applied by the same row gathers as the fine one.  Coarse matrices are the
// Galerkin products P^T A P of the piecewise-constant prolongation P, formed
// once per time step from the assembled matrix; the smoother is weighted
// Jacobi.  One application w = M r:
//   level l, right side b: x = 0; nu sweeps x += omega (b - A x) / diag;
//   b_{l+1} = the residual b - A x summed over each block; the cycle on
//   level l + 1; x += its result on every cell of the block; nu sweeps.
//   The coarsest level (at most 512 cells, or a side shorter than 3): nu_c
//   sweeps from x = 0.
// Every sum is taken in the order of the sequential definition (a block's
// cells in ascending index, a row's entries in face order), so each level's
// matrix and each application equal the sequential cycle's bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "lf_solver.h"

namespace lf {

constexpr int kAmgNu = 2;             // sweeps before and after the coarse correction
constexpr int kAmgNuC = 4;            // sweeps on the coarsest level
constexpr double kAmgOmega = 0.8;     // Jacobi weight
constexpr int64_t kAmgCoarsest = 512; // a level this small is not coarsened further
constexpr int32_t kAmgMinSide = 3;    // nor one with a side shorter than this
static_assert(kAmgNu >= 1 && kAmgNuC >= 2, "level 0's last sweep must not be its first");

struct AmgBox {
    int32_t nx, ny, nz;
    int32_t n() const { return nx * ny * nz; }
};

static std::vector<AmgBox> amg_boxes(const lf_mesh *m) {
    std::vector<AmgBox> v{{m->box_nx, m->box_ny, m->box_nz}};
    for (;;) {
        const AmgBox b = v.back();
        if (static_cast<int64_t>(b.n()) <= kAmgCoarsest || std::min({b.nx, b.ny, b.nz}) < kAmgMinSide) break;
        v.push_back({(b.nx + 1) / 2, (b.ny + 1) / 2, (b.nz + 1) / 2});
    }
    return v;
}

void carve_amg(Carver &cv, const lf_mesh *m, lf_problem *P) {
    const std::vector<AmgBox> boxes = amg_boxes(m);
    double *t1 = cv.take<double>(static_cast<size_t>(m->N));
    double *t2 = cv.take<double>(static_cast<size_t>(m->N));
    std::vector<AmgLevel> lv;
    for (size_t l = 1; l < boxes.size(); ++l) {
        AmgLevel a;
        a.nx = boxes[l].nx;
        a.ny = boxes[l].ny;
        a.nz = boxes[l].nz;
        a.n = boxes[l].n();
        const size_t n = static_cast<size_t>(a.n);
        a.coef = cv.take<double>(3 * n);
        a.diag = cv.take<double>(n);
        a.b = cv.take<double>(n);
        a.xa = cv.take<double>(n);
        a.xb = cv.take<double>(n);
        lv.push_back(a);
    }
    if (P) {
        P->amg = lv;
        P->amg_t1 = t1;
        P->amg_t2 = t2;
    }
}

static BandLayout<3> box_layout(int32_t nx, int32_t ny, int32_t nz) {
    BandLayout<3> L;
    L.n = nx * ny * nz;
    L.d[0] = 1;
    L.d[1] = nx;
    L.d[2] = nx * ny;
    L.mag_sf = nullptr;
    L.delta = nullptr;
    return L;
}

// first sweep, from x = 0 (A x = 0): x = 0 + omega ((b - 0) / diag)
__global__ void __launch_bounds__(kCellBlock)
k_amg_first(int32_t n, const double *__restrict__ b, const double *__restrict__ diag, double *__restrict__ x,
            const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c < n) x[c] = 0.0 + kAmgOmega * ((b[c] - 0.0) / diag[c]);
}

// y = x + omega ((b - A x) / diag), A x with the diagonal term first; kDot
// (level 0's last sweep, y = w, b = r): also the partial sums of w.r
template <bool kDot>
__global__ void __launch_bounds__(kCellBlock)
k_amg_sweep(SolverParams sp, BandLayout<3> L, const double *__restrict__ diag, const double *__restrict__ coef,
            const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ y,
            double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    double acc[1] = {0.0};
    if (c < L.n) {
        const double dc = diag[c], xc = x[c], bc = b[c];
        const double ax = layout_dot(L, c, coef, x, dc * xc);
        const double v = xc + kAmgOmega * ((bc - ax) / dc);
        y[c] = v;
        acc[0] = v * bc;
    }
    if (kDot) {
        const int slots[1] = {kPartWr};
        write_partials<1>(part, sp.grid, slots, acc);
    }
}

// coarse right side: per block, the residual b - A x of its cells (ascending)
__global__ void __launch_bounds__(kCellBlock)
k_amg_restrict(BandLayout<3> F, int32_t fnx, int32_t fny, int32_t fnz, const double *__restrict__ diag,
               const double *__restrict__ coef, const double *__restrict__ b, const double *__restrict__ x,
               int32_t cnx, int32_t cny, int32_t cn, double *__restrict__ bc, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t I = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (I >= cn) return;
    const int32_t ix = I % cnx, iy = (I / cnx) % cny, iz = I / (cnx * cny);
    double acc = 0.0;
    for (int e = 0; e < 2; ++e) {
        const int32_t fz = 2 * iz + e;
        if (fz >= fnz) break;
        for (int bb = 0; bb < 2; ++bb) {
            const int32_t fy = 2 * iy + bb;
            if (fy >= fny) break;
            for (int a = 0; a < 2; ++a) {
                const int32_t fx = 2 * ix + a;
                if (fx >= fnx) break;
                const int32_t c = fx + fnx * (fy + fny * fz);
                const double dc = diag[c];
                const double ax = layout_dot(F, c, coef, x, dc * x[c]);
                acc += b[c] - ax;
            }
        }
    }
    bc[I] = acc;
}

// x += the coarse result of the cell's block
__global__ void __launch_bounds__(kCellBlock)
k_amg_prolong(int32_t fnx, int32_t fny, int32_t fn, int32_t cnx, int32_t cny, double *__restrict__ x,
              const double *__restrict__ xc, const PcgState *__restrict__ st) {
    if (st->done) return;
    const int32_t c = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (c >= fn) return;
    const int32_t fx = c % fnx, fy = (c / fnx) % fny, fz = c / (fnx * fny);
    x[c] += xc[fx / 2 + cnx * (fy / 2 + cny * (fz / 2))];
}

// Galerkin coarse matrix of one block: diag = its cells' diagonals (ascending)
// then twice each face inside it (ascending face order: by cell, then +x,
// +y, +z); the coarse face to the next block in direction k = the sum of the
// fine faces crossing to it, owned by the block's cells on that side
// (ascending).  A block at the end of a direction stores 0 there.
__global__ void __launch_bounds__(kCellBlock)
k_amg_galerkin(int32_t fnx, int32_t fny, int32_t fnz, const double *__restrict__ diag,
               const double *__restrict__ coef, int32_t cnx, int32_t cny, int32_t cnz,
               double *__restrict__ cdiag, double *__restrict__ ccoef) {
    const int32_t cn = cnx * cny * cnz;
    const int32_t I = static_cast<int32_t>(blockIdx.x) * kCellBlock + static_cast<int32_t>(threadIdx.x);
    if (I >= cn) return;
    const int64_t fn = static_cast<int64_t>(fnx) * fny * fnz;
    const int32_t ix = I % cnx, iy = (I / cnx) % cny, iz = I / (cnx * cny);
    // cells of the block per direction (1 at the end of an odd side)
    const int32_t sx = fnx - 2 * ix < 2 ? 1 : 2, sy = fny - 2 * iy < 2 ? 1 : 2, sz = fnz - 2 * iz < 2 ? 1 : 2;
    double dg = 0.0;
    for (int e = 0; e < sz; ++e)
        for (int bb = 0; bb < sy; ++bb)
            for (int a = 0; a < sx; ++a)
                dg += diag[(2 * ix + a) + fnx * ((2 * iy + bb) + fny * (2 * iz + e))];
    for (int e = 0; e < sz; ++e)
        for (int bb = 0; bb < sy; ++bb)
            for (int a = 0; a < sx; ++a) {
                const int64_t c = (2 * ix + a) + fnx * ((2 * iy + bb) + static_cast<int64_t>(fny) * (2 * iz + e));
                if (a + 1 < sx) dg += 2.0 * coef[c];
                if (bb + 1 < sy) dg += 2.0 * coef[fn + c];
                if (e + 1 < sz) dg += 2.0 * coef[2 * fn + c];
            }
    cdiag[I] = dg;
    // the crossing faces in each direction
    const int32_t span[3] = {sx, sy, sz};
    for (int k = 0; k < 3; ++k) {
        double u = 0.0;
        if (span[k] == 2) {
            for (int e = 0; e < sz; ++e)
                for (int bb = 0; bb < sy; ++bb)
                    for (int a = 0; a < sx; ++a) {
                        const int side = k == 0 ? a : (k == 1 ? bb : e);
                        if (side != 1) continue;
                        const int64_t c =
                            (2 * ix + a) + fnx * ((2 * iy + bb) + static_cast<int64_t>(fny) * (2 * iz + e));
                        u += coef[k * fn + c];
                    }
        }
        ccoef[static_cast<int64_t>(k) * cn + I] = u;
    }
}

static dim3 grid_for(int64_t n) {
    return dim3(static_cast<unsigned>(std::max<int64_t>(1, (n + kCellBlock - 1) / kCellBlock)));
}

// the matrix, right side and work vectors of level l (0: the problem's own)
struct AmgView {
    int32_t nx, ny, nz;
    const double *coef, *diag;
    double *ta, *tb;
};

static AmgView amg_view(const lf_problem *P, size_t l) {
    const lf_mesh *m = P->mesh;
    if (l == 0) return AmgView{m->box_nx, m->box_ny, m->box_nz, P->coef, P->diagB, P->amg_t1, P->amg_t2};
    const AmgLevel &a = P->amg[l - 1];
    return AmgView{a.nx, a.ny, a.nz, a.coef, a.diag, a.xa, a.xb};
}

void launch_amg_galerkin(lf_problem *P, hipStream_t s) {
    for (size_t l = 1; l <= P->amg.size(); ++l) {
        const AmgView f = amg_view(P, l - 1);
        const AmgLevel &c = P->amg[l - 1];
        LF_LAUNCH(P, LF_K_AMG_GALERKIN, s, k_amg_galerkin, grid_for(c.n), dim3(kCellBlock), 0, s, f.nx, f.ny, f.nz,
                  f.diag, f.coef, c.nx, c.ny, c.nz, c.diag, c.coef);
    }
}

// One cycle on level l for the right side b; the result ends in `out` when
// given (level 0: w, with the w.r partials), else in one of the level's work
// vectors, which is returned.
static const double *amg_cycle(lf_problem *P, size_t l, const double *b, double *out, hipStream_t s) {
    const AmgView v = amg_view(P, l);
    const BandLayout<3> L = box_layout(v.nx, v.ny, v.nz);
    const int32_t n = L.n;
    const bool coarsest = l == P->amg.size();
    double *cur = nullptr;
    // the first sweep of a level starts from x = 0; level 0's last one (never
    // its first: two or more sweeps per level) also forms the w.r partials
    auto sweep = [&](double *dst, bool last) {
        if (!cur) {
            LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_first, grid_for(n), dim3(kCellBlock), 0, s, n, b, v.diag, dst,
                      P->state);
        } else if (last && l == 0) {
            LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_sweep<true>, grid_for(n), dim3(kCellBlock), 0, s, P->sp, L,
                      v.diag, v.coef, b, cur, dst, P->part, P->state);
        } else {
            LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_sweep<false>, grid_for(n), dim3(kCellBlock), 0, s, P->sp, L,
                      v.diag, v.coef, b, cur, dst, P->part, P->state);
        }
        cur = dst;
    };
    auto other = [&]() { return cur == v.ta ? v.tb : v.ta; };
    if (coarsest) {
        for (int k = 0; k < kAmgNuC; ++k) {
            const bool last = k == kAmgNuC - 1;
            sweep(last && out ? out : other(), last);
        }
        return cur;
    }
    for (int k = 0; k < kAmgNu; ++k) sweep(other(), false);
    AmgLevel &c = P->amg[l];
    LF_LAUNCH(P, LF_K_AMG_RESTRICT, s, k_amg_restrict, grid_for(c.n), dim3(kCellBlock), 0, s, L, v.nx, v.ny, v.nz,
              v.diag, v.coef, b, cur, c.nx, c.ny, c.n, c.b, P->state);
    const double *xc = amg_cycle(P, l + 1, c.b, nullptr, s);
    LF_LAUNCH(P, LF_K_AMG_PROLONG, s, k_amg_prolong, grid_for(n), dim3(kCellBlock), 0, s, v.nx, v.ny, n, c.nx,
              c.ny, cur, xc, P->state);
    for (int k = 0; k < kAmgNu; ++k) {
        const bool last = k == kAmgNu - 1;
        sweep(last && out ? out : other(), last);
    }
    return cur;
}

void launch_amg_cycle(lf_problem *P, hipStream_t s) { amg_cycle(P, 0, P->r, P->w, s); }

}  // namespace lf
