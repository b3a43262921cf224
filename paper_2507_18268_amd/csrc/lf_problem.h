// Problem handle: one mesh + boundary conditions + DT + dt + solver options.
#pragma once

#include "lf_internal.h"

namespace lf {

// Slots of the per-workgroup partial sums (deterministic two-stage reductions:
// every cell-parallel workgroup writes its partial, a one-workgroup kernel
// sums them in a fixed order).
enum PartialSlot : int {
    kPartSumX = 0,   // sum of x0 (mean for the normalisation factor)
    kPartSumR = 1,   // sum |r|
    kPartNf = 2,     // sum |A x0 - pA| + |b - pA|
    kPartWr = 3,     // sum w.r
    kPartPq = 4,     // sum p.Ap
    kPartSumR32 = 5, // precision form, at a pass start: sum |r| of the inner solve's residual
    kPartWr32 = 6,   //   (sum s_c |rs_c|, rs its scaled form) and sum rs.rs,
    kPartRp32 = 7,   //   and sum rs.p with the previous pass's last direction p
    kNumPart = 8
};

// Solver state on the device.  Written only by the one-workgroup reduction
// kernels; the cell-parallel kernels only read it.
struct PcgState {
    double nf;            // normalisation factor
    double res0;          // initial normalised residual
    double res;           // current normalised residual
    double wArA;          // w.r of the current iteration
    double alpha;         // step length of the current iteration
    double beta;          // direction coefficient of the next iteration
    double x_avg;         // mean of x0
    double gamma;         // mixed: weight of rs in the first direction of a continued pass
    int32_t n_iter;
    int32_t done;
    int32_t converged;
    int32_t singular;
    int32_t nonfinite;
    int32_t flag;         // scratch flag (input checks)
    // mixed precision: inner FP32 solve of one refinement pass
    double inner_target;  // stop when the inner residual's L1 norm <= this
    int32_t inner_done;
    int32_t inner_iter;   // iterations of the current pass
    int32_t n_outer;      // refinement passes
    int32_t inner_pend;   // y += alpha p of the last inner update not applied yet
    int32_t inner_cont;   // this pass continues the previous one's CG (keeps its direction)
    int32_t pad3;
    // small solves (decisions taken inside the update and direction kernels):
    // wArA, n_iter and converged as the iteration's update found them
    double wArA_prev;
    int32_t n_iter_prev;
    int32_t conv_prev;
};

// Block walk of a box's band layout (the tiles, lanes and rows are described
// with the walk itself in lf_kernels.h)
// lines and planes of a tile by the rows a lane holds: two planes for the
// FP64 walk (W = 2), one for the FP32 walk (W = 4), whose eight-row groups
// ran 12% faster that way at 256^3 (the FP64 walk 2% slower)
constexpr int bw_lines(int) { return 2; }
constexpr int bw_planes(int W) { return W == 2 ? 2 : 1; }
constexpr int kBwBlock = 256;       // threads of a block-walk workgroup
// a box takes the block walk from this many of its workgroups (4.2 M cells and
// up) whatever the row walk's workgroup count
constexpr int kBoxMinBlocks = 2048;

// host-side plan of a block walk with W x-adjacent rows per lane
struct BoxWalk {
    int32_t hx;        // threads per tile (nx / W)
    int32_t ny;        // lines per plane
    int32_t nyb;       // tiles per plane column (ceil(ny / lines))
    int32_t ntiles;    // nyb ceil(nz / planes)
    int32_t blocks;    // workgroups of kBwBlock threads
};

inline bool box_walk_plan(int32_t n, int32_t K, const int32_t *d, int32_t W, BoxWalk *bw) {
    if (K != 3 || W < 1 || n <= 0 || n % W != 0 || d[0] != 1 || d[1] < W || d[1] % W != 0 || d[2] % d[1] != 0)
        return false;
    const int64_t hx = d[1] / W, ny = d[2] / d[1], nz = (static_cast<int64_t>(n) + d[2] - 1) / d[2];
    const int64_t ty = bw_lines(W), tz = bw_planes(W);
    const int64_t nyb = (ny + ty - 1) / ty, ntiles = nyb * ((nz + tz - 1) / tz);
    const int64_t blocks = (ntiles * hx + kBwBlock - 1) / kBwBlock;
    if (ntiles > INT32_MAX || blocks > INT32_MAX) return false;
    *bw = BoxWalk{static_cast<int32_t>(hx), static_cast<int32_t>(ny), static_cast<int32_t>(nyb),
                  static_cast<int32_t>(ntiles), static_cast<int32_t>(blocks)};
    return true;
}

constexpr int kMaxGraphLog = 6;   // largest captured block: 64 iterations
// FP64 solves with the diagonal preconditioner whose product and update write
// at most this many partials per slot take the iteration's decisions inside
// the update and direction kernels (every workgroup sums the partials)
constexpr int32_t kFoldPartials = 512;

struct SolverParams {
    double tol, rel_tol;
    int32_t max_iter, min_iter;
    int32_t n;            // cells
    int32_t grid;         // workgroups of a cell-parallel launch (= partials per slot)
    int32_t grid_mx;      // workgroups of an FP32 inner-solve launch (kMxRows rows per thread)
    int32_t n_red;        // DIC: first black cell
    int32_t max_outer;    // mixed: refinement passes cap
    int32_t grid_amul;    // workgroups of the FP64 Amul launch (= its p.q partials)
    int32_t grid_mx_amul; // workgroups of the FP32 inner Amul launch (= its p.q partials)
    int32_t inner_restart;// mixed: 1 restarts the inner CG at every refinement pass
    int32_t grid_upd;     // workgroups of the FP64 update launch (= its |r| and w.r partials)
    double inner_tol;     // mixed: relative reduction of each inner solve
};

}  // namespace lf

namespace lf {
struct StepDriver;

// One coarse level of the multigrid preconditioner: a box of nx x ny x nz
// cells numbered i + nx (j + ny k) whose matrix is kept in the band layout
// (offsets 1, nx, nx*ny; slot k*n + c holds the face (c, c + d_k), 0 where
// there is none); b its right side, xa and xb its iterates.
struct AmgLevel {
    int32_t n = 0, nx = 0, ny = 0, nz = 0;
    double *coef = nullptr;      // [3n]
    double *diag = nullptr;      // [n]
    double *b = nullptr, *xa = nullptr, *xb = nullptr;   // [n]
};
}  // namespace lf

struct lf_problem {
    const lf_mesh *mesh = nullptr;
    lf::StepDriver *async = nullptr;           // lf_step_begin's run (null when none has started)
    lf_group *group = nullptr;                 // the group running it (lf_group_add .. finished)
    lf_solver_opts opts{};
    double DT = 0, dt = 0;
    hipStream_t stream = nullptr;
    lf::SolverParams sp{};
    std::vector<lf_patch_bc> bcs;
    // device arrays (caller workspace)
    int32_t *patch_type = nullptr;
    double *patch_value = nullptr;
    double *T = nullptr;                       // [N] the field; PCG solves in place
    double *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr, *w = nullptr, *rD = nullptr;
    double *diag = nullptr, *source = nullptr, *diagB = nullptr, *srcB = nullptr;
    bool banded = false;                       // coefficients in the band layout
    bool rb = false;                           // coefficients in the two-colour band layout (DIC)
    bool walk = false;                         // FP64 Amul by the row walk (bands >= 2, large meshes)
    bool box = false;                          // FP64 products by the block walk (box band layouts, with walk)
    lf::BoxWalk bw{};                          // its plan (2 rows per lane)
    bool box32 = false;                        // the FP32 inner product too (mixed; 4 rows per lane)
    lf::BoxWalk bw32{};
    bool rb2 = false;                          // DIC's kernels on the two-colour layout: two pairs per lane
    bool sumx_valid = false;                   // the part array holds the partial sums of the current T
                                               // (written by the FP64 commit; any other write of T clears it)
    bool fold = false;                         // small diagonal FP64 solves: the iteration's reductions folded
                                               // into the update and direction kernels
    bool scaled = false;                       // diagonal FP64 solves on the block walk (not folded): CG on
                                               // the Jacobi-scaled matrix; during a solve rD holds sqrt(diagB),
                                               // r, p, q the scaled vectors and w the scaled iterate
    double *coefS = nullptr;                   // [3N] its off-diagonal band coefficients
    // multigrid preconditioner: coarse levels 1.. (level 0 is the problem's own
    // band matrix) and two work vectors of level 0
    std::vector<lf::AmgLevel> amg;
    double *amg_t1 = nullptr, *amg_t2 = nullptr;   // [N]
    // per level (0: the problem's box): its block walk, and 0 none, 1 the
    // sweeps walk, 2 the restriction too (all sides even)
    std::vector<lf::BoxWalk> amg_bw;
    std::vector<int8_t> amg_walk;
    double *upper = nullptr;                   // [F] face order (test hook copy)
    double *coef = nullptr;                    // [n_entries] row layout or [n_bands N] bands
    double *int_coeff = nullptr, *bou_coeff = nullptr;
    double *Tb = nullptr;                      // [B] boundary-face values (output staging)
    // non-orthogonal meshes: the gradient of T at assembly (solver order) and
    // the Laplacian's explicit source built from it
    bool nonorth = false;
    double *grad3 = nullptr;                   // [3N]: by component on band-form meshes, else xyz per cell
    double *lap_src = nullptr;                 // [N]
    double *T_old = nullptr;                   // [N] T at the start of the step (corrector passes)
    double *snb = nullptr;                     // [B] normal gradient of T on the boundary faces
                                               // (lf_problem_grad; meshes with gradient geometry)
    double *part = nullptr;                    // [kNumPart][grid]
    lf::PcgState *state = nullptr;
    // mixed precision (FP32 inner solve)
    float *coef32 = nullptr, *diag32 = nullptr, *rD32 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    float *sig32 = nullptr;                    // multi-kernel precision form: sqrt(diagB) in FP32
    // host side
    lf::PcgState *h_state = nullptr;           // pinned
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t g_iter[lf::kMaxGraphLog + 1] = {};   // 2^i PCG iterations
    hipGraphExec_t g_inner[lf::kMaxGraphLog + 1] = {};  // 2^i inner FP32 iterations
    int32_t last_iters = 0;
    // precision form, for sizing the iteration blocks: inner iterations of
    // each refinement pass and the number of passes of the last step
    static constexpr int kPassTrack = 8;
    int32_t last_inner[kPassTrack] = {};
    int32_t last_outer = 0;
    bool assembled = false;
    bool scaled32 = false;                     // mixed: the inner solve's FP32 coefficients are formed
    size_t ws_bytes = 0;
    // per-kernel device timing (diagnostics)
    bool prof_on = false;
    int64_t prof_ticks = 0;                    // lead time of the timing spin (wall-clock ticks)
    double prof_ms[LF_NUM_KERNEL_CLASSES] = {};
    int64_t prof_n[LF_NUM_KERNEL_CLASSES] = {};
    struct ProfRec { int cls; hipEvent_t a, b; };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
};

namespace lf {
// Records an event pair around one kernel launch when timing is on and the
// launch goes to the handle's own stream (never inside a graph capture).
struct ProfScope {
    lf_problem *P;
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr;
    bool on;
    hipEvent_t get() {
        if (P->ev_used == P->ev_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            P->ev_pool.push_back(e);
        }
        return P->ev_pool[P->ev_used++];
    }
    ProfScope(lf_problem *P_, int cls_, hipStream_t s_) : P(P_), cls(cls_), s(s_) {
        on = P->prof_on && s == P->stream;
        if (on) {
            a = get();
            on = a && hipEventRecord(a, s) == hipSuccess;
        }
    }
    ~ProfScope() {
        if (!on) return;
        hipEvent_t b = get();
        if (b && hipEventRecord(b, s) == hipSuccess) P->prof_pending.push_back({cls, a, b});
    }
};
// accumulate the recorded pairs (call after the stream has been synchronised)
void prof_flush(lf_problem *P);
// when timing: a short GPU-side wait ahead of the launches that follow
void prof_lead(lf_problem *P, hipStream_t s);
}  // namespace lf

#define LF_LAUNCH(P, cls, s, ...)                  \
    do {                                           \
        ::lf::ProfScope ps_((P), (cls), (s));       \
        hipLaunchKernelGGL(__VA_ARGS__);           \
    } while (0)
