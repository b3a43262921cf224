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
// a level takes the block walk from this many workgroups on (about 2 M cells;
// on smaller levels, whose launches are latency-bound, the one-row kernels
// finish sooner)
constexpr int32_t kAmgWalkMinBlocks = 1024;
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

static void plan_amg_walks(lf_problem *P);

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
        plan_amg_walks(P);
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

// ---------------------------------------------------------------------------
// The same steps by the block walk of a box level (x-lines of even length: two
// rows per lane, 2 lines x 2 planes per thread, as the solver's product): each
// row's A x is the one-row kernels' sum term for term, so every result is
// bitwise the same.
// ---------------------------------------------------------------------------

// the first sweep's values (x = 0 + omega (b - 0) / diag), formed where the
// walk asks for x
struct AmgFirstX {
    const double *__restrict__ b;
    const double *__restrict__ diag;
    __device__ __forceinline__ Lanes<double, 2> vec(int64_t i) const {
        const Lanes<double, 2> bb = lanes_load<double, 2>(b, i), dd = lanes_load<double, 2>(diag, i);
        Lanes<double, 2> r;
#pragma unroll
        for (int w = 0; w < 2; ++w) r.v[w] = 0.0 + kAmgOmega * ((bb.v[w] - 0.0) / dd.v[w]);
        return r;
    }
    __device__ __forceinline__ double one(int64_t i) const { return 0.0 + kAmgOmega * ((b[i] - 0.0) / diag[i]); }
};

// Quotient by a fixed divisor d >= 1 for 0 <= i < 2^31 by a multiply and a
// shift (Granlund and Montgomery 1994): with s = ceil(log2 d) and
// m = floor(2^(32+s) / d) + 1, floor(i m / 2^(32+s)) = floor(i / d), since
// m d - 2^(32+s) lies in (0, d] and i < 2^32.
struct FastDiv {
    uint64_t m;
    int32_t sh;
};

inline FastDiv fast_div(uint32_t d) {
    int32_t s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    return FastDiv{((uint64_t(1) << (32 + s)) / d) + 1, 32 + s};
}

__device__ __forceinline__ int64_t fdiv(int64_t i, const FastDiv &f) {
    return static_cast<int64_t>((static_cast<uint64_t>(i) * f.m) >> f.sh);
}

// the prolonged iterate x + (the coarse result of the cell's block), formed
// where the walk asks for x (a lane's two cells lie in one block: x-lines of
// even length)
struct AmgProlongX {
    const double *__restrict__ x;
    const double *__restrict__ xc;
    int64_t nx, ny, cnx, cny;
    FastDiv dx, dy;
    __device__ __forceinline__ int64_t block(int64_t i) const {
        const int64_t t = fdiv(i, dx), fx = i - t * nx, fz = fdiv(t, dy), fy = t - fz * ny;
        return (fx >> 1) + cnx * ((fy >> 1) + cny * (fz >> 1));
    }
    __device__ __forceinline__ Lanes<double, 2> vec(int64_t i) const {
        Lanes<double, 2> r = lanes_load<double, 2>(x, i);
        const double a = xc[block(i)];
#pragma unroll
        for (int w = 0; w < 2; ++w) r.v[w] += a;
        return r;
    }
    __device__ __forceinline__ double one(int64_t i) const { return x[i] + xc[block(i)]; }
};

// y = x + omega ((b - A x) / diag) with x from the source: the level's
// iterate, (AmgFirstX) the first sweep's values, so that the launch does the
// level's first two sweeps, or (AmgProlongX) the iterate with the coarse
// correction added, so that it also does the prolongation.  kDot (level 0's
// last sweep, y = w, b = r): the partial sums of w.r, one per workgroup, and
// zeros in the further entries of the slot up to the cell grid's count, which
// the reduction reads
template <class XS, bool kDot>
__global__ void __launch_bounds__(kBwBlock)
k_amg_sweep_box(SolverParams sp, BandLayout<3> L, BoxWalk bw, const double *__restrict__ diag,
                const double *__restrict__ coef, const double *__restrict__ b, XS x, double *__restrict__ y,
                double *__restrict__ part, const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    double acc[1] = {0.0};
    box_walk_xs<double, 2, false, false>(L, bw, diag, coef, x, [&](int64_t c, const R &ax, const R &xc, const R &dg) {
        const R bc = lanes_load<double, 2>(b, c);
        R v;
#pragma unroll
        for (int w = 0; w < 2; ++w) v.v[w] = xc.v[w] + kAmgOmega * ((bc.v[w] - ax.v[w]) / dg.v[w]);
        *reinterpret_cast<typename R::vec *>(y + c) = typename R::vec{v.v[0], v.v[1]};
        if (kDot) {
            acc[0] += v.v[0] * bc.v[0];
            acc[0] += v.v[1] * bc.v[1];
        }
    });
    if (kDot) {
        const int slots[1] = {kPartWr};
        write_partials<1, kBwBlock>(part, sp.grid, slots, acc);
        if (threadIdx.x == 0)
            for (int64_t j = bw.blocks + static_cast<int64_t>(blockIdx.x); j < sp.grid; j += bw.blocks)
                part[static_cast<int64_t>(kPartWr) * sp.grid + j] = 0.0;
    }
}

// k_amg_restrict on a level whose sides are all even: the walk's tiles are the
// 2 x 2 x 2 blocks (tile thread i is coarse cell i); the block's residuals are
// summed in the one-row kernel's order (z, then y, then x)
__global__ void __launch_bounds__(kBwBlock)
k_amg_restrict_box(BandLayout<3> L, BoxWalk bw, const double *__restrict__ diag, const double *__restrict__ coef,
                   const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ bc,
                   const PcgState *__restrict__ st) {
    if (st->done) return;
    typedef Lanes<double, 2> R;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBwBlock + threadIdx.x;
    R res[2][2];
    // the walk visits a tile's rows line by line, within a line plane by plane
    int call = 0;
    box_walk<double, 2, false, false>(L, bw, diag, coef, x, [&](int64_t c, const R &ax, const R &, const R &) {
        const R bb = lanes_load<double, 2>(b, c);
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
                if (2 * jj + kk == call)
#pragma unroll
                    for (int w = 0; w < 2; ++w) res[jj][kk].v[w] = bb.v[w] - ax.v[w];
        ++call;
    });
    if (i >= static_cast<int64_t>(bw.ntiles) * bw.hx) return;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) acc += res[bb][e].v[a];
    bc[i] = acc;
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

// the block walk of each level (index 0: the problem's own box) where its
// x-lines have even length, and whether its sides are all even (then the
// restriction to the next level runs on it too)
static void plan_amg_walks(lf_problem *P) {
    const lf_mesh *m = P->mesh;
    const size_t nl = P->amg.size() + 1;
    P->amg_bw.assign(nl, BoxWalk{});
    P->amg_walk.assign(nl, 0);
    for (size_t l = 0; l < nl; ++l) {
        const int32_t nx = l == 0 ? m->box_nx : P->amg[l - 1].nx, ny = l == 0 ? m->box_ny : P->amg[l - 1].ny;
        const int32_t nz = l == 0 ? m->box_nz : P->amg[l - 1].nz;
        const int32_t d[3] = {1, nx, nx * ny};
        BoxWalk bw;
        // LF_WALK_ON takes it on every level that allows it (tests), LF_WALK_OFF on none
        const int32_t wo = P->opts.amul_walk;
        if (wo != LF_WALK_OFF && nx % 2 == 0 && box_walk_plan(nx * ny * nz, 3, d, 2, &bw) &&
            (wo == LF_WALK_ON || bw.blocks >= kAmgWalkMinBlocks) && bw.blocks <= P->sp.grid) {
            P->amg_bw[l] = bw;
            P->amg_walk[l] = (ny % 2 == 0 && nz % 2 == 0) ? 2 : 1;
        }
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
    const int walk = P->amg_walk[l];
    const BoxWalk bw = P->amg_bw[l];
    const dim3 wgrid(static_cast<unsigned>(std::max<int32_t>(1, bw.blocks)));
    // the first sweep of a level starts from x = 0; level 0's last one (never
    // its first: two or more sweeps per level) also forms the w.r partials.
    // On a walked level the first two sweeps are one launch, the first sweep
    // after the coarse correction also adds it (prolongation), and the other
    // sweeps take the walk too.
    const double *pending = nullptr;   // coarse result not yet added to cur
    const AmgLevel *cl = coarsest ? nullptr : &P->amg[l];
    auto sweep = [&](double *dst, bool last, bool can_pair) {
        const bool dot = last && l == 0;
        if (!cur && walk && can_pair) {
            LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, (k_amg_sweep_box<AmgFirstX, false>), wgrid, dim3(kBwBlock), 0, s, P->sp,
                      L, bw, v.diag, v.coef, b, AmgFirstX{b, v.diag}, dst, P->part, P->state);
            cur = dst;
            return 2;
        }
        if (!cur) {
            LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_first, grid_for(n), dim3(kCellBlock), 0, s, n, b, v.diag, dst,
                      P->state);
        } else if (walk && pending) {
            const AmgProlongX px{cur, pending, v.nx, v.ny, cl->nx, cl->ny, fast_div(static_cast<uint32_t>(v.nx)),
                                 fast_div(static_cast<uint32_t>(v.ny))};
            if (dot)
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, (k_amg_sweep_box<AmgProlongX, true>), wgrid, dim3(kBwBlock), 0, s,
                          P->sp, L, bw, v.diag, v.coef, b, px, dst, P->part, P->state);
            else
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, (k_amg_sweep_box<AmgProlongX, false>), wgrid, dim3(kBwBlock), 0, s,
                          P->sp, L, bw, v.diag, v.coef, b, px, dst, P->part, P->state);
        } else if (walk) {
            if (dot)
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, (k_amg_sweep_box<MemX<double, 2>, true>), wgrid, dim3(kBwBlock), 0,
                          s, P->sp, L, bw, v.diag, v.coef, b, MemX<double, 2>{cur}, dst, P->part, P->state);
            else
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, (k_amg_sweep_box<MemX<double, 2>, false>), wgrid, dim3(kBwBlock), 0,
                          s, P->sp, L, bw, v.diag, v.coef, b, MemX<double, 2>{cur}, dst, P->part, P->state);
        } else {
            if (pending)
                LF_LAUNCH(P, LF_K_AMG_PROLONG, s, k_amg_prolong, grid_for(n), dim3(kCellBlock), 0, s, v.nx, v.ny, n,
                          cl->nx, cl->ny, cur, pending, P->state);
            if (dot)
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_sweep<true>, grid_for(n), dim3(kCellBlock), 0, s, P->sp, L,
                          v.diag, v.coef, b, cur, dst, P->part, P->state);
            else
                LF_LAUNCH(P, LF_K_AMG_SMOOTH, s, k_amg_sweep<false>, grid_for(n), dim3(kCellBlock), 0, s, P->sp, L,
                          v.diag, v.coef, b, cur, dst, P->part, P->state);
        }
        pending = nullptr;
        cur = dst;
        return 1;
    };
    auto other = [&]() { return cur == v.ta ? v.tb : v.ta; };
    if (coarsest) {
        for (int k = 0; k < kAmgNuC;) {
            // the last sweep writes `out`: a fused first pair must end before it
            const bool last = k == kAmgNuC - 1;
            k += sweep(last && out ? out : other(), last, k + 2 < kAmgNuC);
        }
        return cur;
    }
    for (int k = 0; k < kAmgNu;) k += sweep(other(), false, k + 2 <= kAmgNu);
    AmgLevel &c = P->amg[l];
    if (walk == 2)
        LF_LAUNCH(P, LF_K_AMG_RESTRICT, s, k_amg_restrict_box, wgrid, dim3(kBwBlock), 0, s, L, bw, v.diag, v.coef, b,
                  cur, c.b, P->state);
    else
        LF_LAUNCH(P, LF_K_AMG_RESTRICT, s, k_amg_restrict, grid_for(c.n), dim3(kCellBlock), 0, s, L, v.nx, v.ny,
                  v.nz, v.diag, v.coef, b, cur, c.nx, c.ny, c.n, c.b, P->state);
    pending = amg_cycle(P, l + 1, c.b, nullptr, s);
    for (int k = 0; k < kAmgNu; ++k) {
        const bool last = k == kAmgNu - 1;
        sweep(last && out ? out : other(), last, false);
    }
    return cur;
}

void launch_amg_cycle(lf_problem *P, hipStream_t s) { amg_cycle(P, 0, P->r, P->w, s); }

}  // namespace lf
