/*
 * lapfoam.h -- C interface of the MI355X (gfx950) laplacianFoam hot path.
 *
 * The library advances  dT/dt - div(DT grad T) = 0  (Eq. 1 of the paper with an
 * empty source term) by implicit-Euler time steps on a finite-volume mesh given
 * in OpenFOAM face addressing (Section 4: per internal face an owner and a
 * neighbour cell, face area vector pointing owner -> neighbour; boundary faces
 * grouped into patches).  Each step assembles
 *      TEqn = fvm::ddt(T) - fvm::laplacian(DT, T)            (Listing 1)
 * into an LDU matrix (diag, upper, lower = upper, source and per-boundary-face
 * internal / boundary coefficients) and solves it with the preconditioned
 * conjugate gradient method (Sections 5.1 and 6: PCG with the diagonal
 * preconditioner; a DIC preconditioner on red-black numbered meshes is also
 * offered).  Cell-parallel loops use the atomic-free "list of lists"
 * addressing of Section 5.2 (ownerStart / losort / losortStart and the
 * boundary face lists of each cell), built on the GPU.
 *
 * Conventions (all entry points):
 *  - Every function returns an lf_status; 0 is success.  On error nothing
 *    observable is half-written unless stated, and lf_last_error() returns a
 *    message (per thread, valid until the next failing call on that thread).
 *  - Device memory comes only from the caller: each handle lives in a
 *    caller-owned device workspace whose exact size the *_workspace_bytes
 *    functions return.  The library never allocates device memory, so a
 *    caller can budget HBM exactly.  The workspace must stay allocated and
 *    untouched until the handle is destroyed.  Workspaces must be 256-byte
 *    aligned.
 *  - Host arrays passed in are read during the call only; the caller keeps
 *    ownership.
 *  - `stream` is a hipStream_t (passed as void*; NULL = the default stream).
 *    All device work of a handle is ordered on the stream given at creation.
 *  - Handles are not thread-safe; distinct handles may be used from distinct
 *    threads.  Calls that overlap on one handle are undefined.
 *  - Integers are int32 (cell and face counts below 2^31), reals IEEE binary64
 *    unless stated.
 */
#ifndef LAPFOAM_H
#define LAPFOAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lf_status;
#define LF_OK 0
#define LF_EINVAL (-1)      /* bad argument (NULL, negative size, dt <= 0, ...) */
#define LF_EMESH (-2)       /* mesh fails validation (see lf_mesh_create) */
#define LF_ENOMEM (-3)      /* workspace too small or misaligned; host allocation failed */
#define LF_EBUDGET (-4)     /* batch: request does not fit the device-memory budget */
#define LF_EDEVICE (-5)     /* a HIP runtime call failed */
#define LF_ESTATE (-6)      /* call not valid in the handle's current state */
#define LF_ENONFINITE (-7)  /* a non-finite value appeared in the solve */

#define LF_BC_ZERO_GRADIENT 0
#define LF_BC_FIXED_VALUE 1

#define LF_PC_DIAGONAL 0   /* w = r / diag (stored as reciprocal, Section 6) */
#define LF_PC_DIC 1        /* diagonal incomplete Cholesky; needs a two-colour
                              numbering: every face's owner < every face's
                              neighbour (all "red" cells before all "black") */
#define LF_PC_AMG 2        /* aggregation multigrid V-cycle (FP64, meshes with
                              the box form: see lf_problem_create) */

#define LF_LAYOUT_AUTO 0   /* bands when the mesh has a band form for the
                              preconditioner (diagonal or multigrid: the band
                              form; DIC: the two-colour band form), else rows */
#define LF_LAYOUT_ROWS 1   /* sliced row layout from the lists of lists: any
                              mesh; each coefficient stored in both its rows */
#define LF_LAYOUT_BANDS 2  /* band layout: meshes whose internal faces take at
                              most 4 distinct offsets neighbour - owner (a
                              structured numbering), with the diagonal or
                              multigrid preconditioner; with DIC, the two-colour
                              band form (a box numbered red cells first, then
                              black, each colour in natural order, x-lines of
                              even length): each face's coefficient stored once
                              at its red cell's direction slot.  Each
                              coefficient stored once, no column indices */

#define LF_WALK_AUTO 0     /* matrix-vector products of a band layout with two
                              or more bands (the FP64 solve's, and the inner
                              FP32 solve's of LF_PREC_MIXED) by the row walk
                              when the mesh fills the GPU with it (at least
                              2048 workgroups of 512 threads, 8 rows each),
                              else one row per thread; the FP64 products of a
                              box then take the block walk
                              (lf_problem_amul_walk), and so they do on any
                              box that gives the block walk at least 2048
                              workgroups of 256 threads (4.2 M cells and up) */
#define LF_WALK_ON 1       /* the row walk whenever the layout allows it (tests) */
#define LF_WALK_OFF 2      /* always one row per thread */

#define LF_PREC_FP64 0     /* everything in binary64 */
#define LF_PREC_MIXED 1    /* FP64 outer residual and update; inner solve in
                              FP32 (coefficients, vectors, SpMV) with FP64 dot
                              products, alpha and beta: CG on S A S, S =
                              diag(1/sqrt(diag A)), which is the diagonally
                              preconditioned CG of A d = r in exact arithmetic
                              (iterative refinement) */

#define LF_MESH_NON_ORTHOGONAL 1   /* lf_mesh_desc.flags: accept faces that are not
                                      orthogonal to the line joining their cell
                                      centres (skewed cells).  Created with face
                                      centres, such a mesh also holds the
                                      Laplacian's correction vectors, and its
                                      problems apply the explicit non-orthogonal
                                      correction every step (see
                                      lf_problem_create) */

/* Mesh in OpenFOAM face addressing (host pointers). */
typedef struct lf_mesh_desc {
    int32_t n_cells;            /* N >= 1 */
    int32_t n_faces;            /* F >= 0 internal faces */
    int32_t n_patches;          /* P >= 0 */
    int32_t flags;              /* 0 or LF_MESH_NON_ORTHOGONAL */
    const int32_t *owner;       /* [F] owner cell of each internal face */
    const int32_t *neighbour;   /* [F] neighbour cell; owner < neighbour and faces
                                   sorted by (owner, neighbour): upper-triangular order */
    const double *cell_volume;  /* [N] V_c > 0 */
    const double *cell_centre;  /* [3N] C_c, xyz interleaved */
    const double *face_area;    /* [3F] S_f, |S_f| = face area, owner -> neighbour */
    const double *face_centre;  /* [3F] C_f; may be NULL: then the mesh holds no
                                   gradient geometry and lf_grad returns LF_EINVAL */
    const int32_t *patch_start; /* [P+1] boundary faces of patch p are
                                   [patch_start[p], patch_start[p+1]); patch_start[0] = 0 */
    const int32_t *bface_cell;  /* [B] cell of each boundary face, B = patch_start[P] */
    const double *bface_area;   /* [3B] outward S_b */
    const double *bface_centre; /* [3B] C_b */
} lf_mesh_desc;

/* Boundary condition of one patch. */
typedef struct lf_patch_bc {
    int32_t type;               /* LF_BC_ZERO_GRADIENT or LF_BC_FIXED_VALUE */
    int32_t reserved;
    double value;               /* fixed value T_b (ignored for zeroGradient) */
} lf_patch_bc;

typedef struct lf_solver_opts {
    double tol;                 /* absolute tolerance on the normalised residual */
    double rel_tol;             /* relative tolerance (0 = off) */
    int32_t max_iter;           /* iteration cap (OpenFOAM default 1000) */
    int32_t min_iter;           /* minimum iterations (default 0) */
    int32_t precond;            /* LF_PC_* */
    int32_t precision;          /* LF_PREC_* */
    int32_t iters_per_check;    /* PCG iterations enqueued between host checks of the
                                   convergence flag; 0 = adaptive */
    int32_t use_graph;          /* 1: replay captured HIP graphs, 0: plain launches */
    double inner_tol;           /* LF_PREC_MIXED: inner FP32 solve stops when its
                                   residual falls by this factor (0 = default 1e-5) */
    int32_t max_outer;          /* LF_PREC_MIXED: refinement passes cap (0 = 50) */
    int32_t layout;             /* LF_LAYOUT_* of the coefficients (default AUTO).
                                   Results do not depend on it beyond the sign
                                   of exact zeros: both layouts sum a row's
                                   entries in the same order */
    int32_t amul_walk;          /* LF_WALK_* (default AUTO).  Both forms give
                                   bitwise the same product; only the order of
                                   the partial sums of p.Ap differs */
    int32_t inner_restart;      /* LF_PREC_MIXED: 0 (default) continues the inner CG
                                   across refinement passes (the true residual
                                   replaces the recurred one, the search direction
                                   is kept); 1 restarts it at every pass */
    int32_t n_nonorth_corr;     /* extra passes of the non-orthogonal corrector loop
                                   per time step, 0..100 (default 0): each pass
                                   assembles TEqn again, its ddt source from T at
                                   the start of the step and its correction from
                                   the latest T, and solves from the latest T.
                                   Used on meshes with non-orthogonal faces only
                                   (elsewhere the correction is zero) */
} lf_solver_opts;

/* Per time step results. */
typedef struct lf_solve_stats {
    double initial_residual;    /* normalised residual of x0 = T_old */
    double final_residual;      /* normalised residual at exit */
    int32_t n_iter;             /* PCG iterations performed (mixed: inner total) */
    int32_t converged;          /* 1 if the last convergence check passed */
    int32_t singular;           /* 1 if |p.Ap| / normFactor < 1e-300 ended the solve */
    int32_t nonfinite;          /* 1 if a NaN/Inf residual or p.Ap appeared */
    int32_t n_outer;            /* mixed: refinement passes (FP64: 1) */
    int32_t reserved;
    double assemble_ms;         /* device time of the assembly (events) */
    double solve_ms;            /* device time of the solve (events) */
} lf_solve_stats;

typedef struct lf_mesh lf_mesh;
typedef struct lf_problem lf_problem;

/* Message of the last failing call on this thread ("" if none). */
const char *lf_last_error(void);

/* Fills *opts with the defaults: tol 1e-9, rel_tol 0, max_iter 1000, min_iter 0,
   diagonal preconditioner, FP64, adaptive checks, graphs on. */
lf_status lf_default_opts(lf_solver_opts *opts);

/* ---- mesh (once per mesh) ------------------------------------------------
 * Validation (LF_EMESH): every owner/neighbour/face cell index in [0, N);
 * owner < neighbour; faces strictly increasing in (owner, neighbour);
 * S.d > 0 for every face (d = C_N - C_P), and unless flags has
 * LF_MESH_NON_ORTHOGONAL every face orthogonal (|S x d| <= 1e-9 |S||d|: such a
 * mesh's problems skip the non-orthogonal correction); boundary faces outward
 * (S_b.(C_b - C_P) > 0); V > 0; unknown flags give LF_EINVAL.
 * With face_centre given, the device copy also holds the gradient's face
 * records (S_f and the interpolation weight w_f, 32 bytes per face) and
 * boundary-face records (S_b and |S_b|), which lf_grad reads.
 * The device copy holds the addressing (Section 5.2 lists of lists: per cell
 * its owned faces, its lower faces in ascending face order, its boundary
 * faces in ascending boundary-face order) and the geometry factors
 * |S_f|, delta_f = 1/max(n.d, 0.05|d|), |S_b|, delta_b = 1/(n.(C_b - C_P)). */
size_t lf_mesh_workspace_bytes(const lf_mesh_desc *desc);
lf_status lf_mesh_create(const lf_mesh_desc *desc, void *dev_workspace, size_t workspace_bytes,
                         void *stream, lf_mesh **out);
lf_status lf_mesh_destroy(lf_mesh *mesh);   /* NULL-safe; does not free the workspace */

/* The mesh's band form: *n_bands distinct offsets neighbour - owner (0 when the
 * faces take more than 4), ascending in offsets[4] (may be NULL; unused
 * entries 0).  Problems on a mesh with n_bands > 0 can use LF_LAYOUT_BANDS. */
lf_status lf_mesh_bands(const lf_mesh *mesh, int32_t *n_bands, int32_t *offsets);

/* Cell order of the solver's arrays.  A mesh without band form and without a
 * two-colour numbering is stored with its cells sorted by the Morton (Z-order)
 * key of their centres (21 bits per axis over the bounding box, ties by cell
 * index), so that a row's neighbours lie near it in memory; every row keeps its
 * entries in the mesh's face order, so each row sum is unchanged.  Fields still
 * cross this interface in the mesh's order.  *reordered = 1 for such a mesh;
 * order[N] (host, may be NULL) receives the mesh cell of each solver row
 * (the identity when not reordered). */
lf_status lf_mesh_cell_order(const lf_mesh *mesh, int32_t *reordered, int32_t *order);

/* Test hook: copies the device addressing to host arrays (any may be NULL):
 * owner_start[N+1] (faces owned by c are [owner_start[c], owner_start[c+1])),
 * losort[F], losort_start[N+1] (faces whose neighbour is c are
 * losort[losort_start[c] .. losort_start[c+1]) in ascending order),
 * bface_start[N+1], bface_list[B] (boundary faces of each cell, ascending). */
lf_status lf_mesh_get_addressing(const lf_mesh *mesh, int32_t *owner_start, int32_t *losort,
                                 int32_t *losort_start, int32_t *bface_start,
                                 int32_t *bface_list);

/* Gauss gradient of a cell field (Section 5.2: calcGrad = linear
 * interpolation to the faces, gradf, then correctBoundaryConditions), for the
 * explicit non-orthogonal correction of the Laplacian:
 *   w_f = |S_f.(C_N - C_f)| / (|S_f.(C_f - C_P)| + |S_f.(C_N - C_f)|) (owner weight),
 *         or 1/2 where that denominator is not above ROOTVSMALL = 1e-150
 *   s_f = w_f (T_P - T_N) + T_N
 *   grad_c = (sum over the faces owned by c of S_f s_f - sum over the faces
 *            whose neighbour is c of S_f s_f + sum over its boundary faces of
 *            S_b Tb_b) / V_c
 *   bgrad_b = grad_P + n (snGrad_b - n.grad_P), n = S_b/|S_b|, P the face cell.
 * One thread takes each cell's faces (lower faces ascending, then owned faces
 * ascending, then boundary faces ascending: the order in which the sequential
 * face loop reaches the cell), from band slots on a mesh with band form, else
 * through the lists of lists, so each result equals, bit for bit, the
 * sequential loop over faces then boundary faces.
 * T[N], Tb[B] (the field's boundary values) and snGrad_b[B] (its normal
 * gradient on the boundary faces) are device inputs in the mesh's cell and
 * boundary-face order; grad[3N] and bgrad[3B] (xyz interleaved, same orders)
 * are device outputs.  bgrad may be NULL (then snGrad_b is not read).  The
 * work is ordered on the mesh's stream and the call returns without waiting.
 * On a mesh kept in Morton order (lf_mesh_cell_order) T is first copied into
 * that order and the gradient is formed in it, both in scratch arrays of the
 * mesh, then gathered back to the mesh's order: calls on one mesh must stay on
 * its stream (not concurrent from several threads).
 * LF_EINVAL: NULL mesh, T, grad, or Tb (B > 0), or snGrad_b with bgrad given;
 * a mesh created without face centres. */
lf_status lf_grad(const lf_mesh *mesh, const double *T, const double *Tb, const double *snGrad_b,
                  double *grad, double *bgrad);

/* lf_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, layouts, ordering and results as lf_grad (bitwise); it calls no
 * hipMalloc, hipFree or allocating library routine.  On a mesh kept in Morton
 * order T is copied into a scratch array that the library holds in static
 * device memory, one per GPU (64 MiB, kept until the process ends), instead of
 * the mesh's workspace; its address on a GPU is looked up on the first call
 * there.  Every call on one GPU shares that array: calls that overlap on one
 * GPU (other streams, other threads, other meshes) race and must be ordered
 * by the caller.  Meshes with band form use no scratch.
 * LF_EINVAL: as lf_grad; a mesh in Morton order with more than 8,388,608
 * cells (the scratch's size); the current device is not the mesh's.
 * LF_EDEVICE: the scratch's address could not be looked up. */
lf_status lf_grad_noalloc(const lf_mesh *mesh, const double *T, const double *Tb, const double *snGrad_b,
                          double *grad, double *bgrad);

/* ---- problem: mesh + boundary conditions + DT + dt + solver ------------- */
size_t lf_problem_workspace_bytes(const lf_mesh *mesh, const lf_solver_opts *opts);
/* bcs[n_patches]; DT >= 0 finite; dt > 0 finite.  LF_PC_DIC on a mesh without
 * the two-colour property returns LF_EINVAL.
 * LF_PC_AMG (Section 7 names an algebraic multigrid library as the better
 * alternative to the diagonal PCG): PCG preconditioned by one V-cycle of
 * aggregation multigrid per iteration.  The mesh must have the box form (band
 * offsets 1, nx, nx*ny of an nx x ny x nz box numbered i + nx (j + ny k),
 * sides >= 2, no face wrapping between lines or planes), FP64, the band
 * layout; else LF_EINVAL.  Level l + 1 aggregates the 2 x 2 x 2 blocks of
 * level l (a side of odd length ends with a one-cell block) while a level has
 * more than 512 cells and every side is 3 or longer; coarse matrices are the
 * Galerkin products P^T A P of the piecewise-constant prolongation, formed
 * after each assembly; the cycle on a level: x = 0, two weighted-Jacobi sweeps
 * x += 0.8 (b - A x) / diag, the residual summed over each block as the next
 * level's right side, its cycle's result added to each cell of the block, two
 * more sweeps; four sweeps from x = 0 on the coarsest level.
 * On a mesh created with LF_MESH_NON_ORTHOGONAL (which then needs face centres,
 * else LF_EINVAL) the Laplacian is the Gauss linear corrected scheme in full
 * (Section 5.1, one pass of the non-orthogonal corrector loop per step): before
 * each assembly the gradient of T (as lf_grad, with T's boundary values) is
 * interpolated to the faces, each face's correction flux
 * (DT |S_f|) (k_f . g_f), k_f = S_f/|S_f| - delta_f (C_N - C_P), is summed per
 * cell in the face loop's order (owned faces +, lower faces -), divided by V_c,
 * and lap_src_c = 0 - V_c div_c is subtracted from TEqn's source.  Such problems
 * are refused by lf_batch_launch.  T starts at 0: set it with lf_set_T before
 * stepping. */
lf_status lf_problem_create(const lf_mesh *mesh, const lf_patch_bc *bcs, double DT, double dt,
                            const lf_solver_opts *opts, void *dev_workspace,
                            size_t workspace_bytes, void *stream, lf_problem **out);
lf_status lf_problem_destroy(lf_problem *problem);  /* NULL-safe */

/* Re-targets an existing problem to new boundary conditions, DT and dt (same
 * mesh, options, workspace and stream; checks as in lf_problem_create).  T is
 * kept: set it with lf_set_T.  Returns after the new values are on the device:
 * when the patch conditions change it synchronises the problem's stream (only
 * that one); DT and dt alone change without waiting.  For callers that solve many
 * problems of one mesh: destroying a problem frees pinned host memory, which
 * waits for the whole device.  Must not be called while a batch launch uses
 * the problem. */
lf_status lf_problem_reset(lf_problem *problem, const lf_patch_bc *bcs, double DT, double dt);

/* The coefficient layout the problem resolved to: LF_LAYOUT_ROWS or
 * LF_LAYOUT_BANDS (never AUTO). */
lf_status lf_problem_layout(const lf_problem *problem, int32_t *layout);

/* How the problem's FP64 matrix-vector products run: 0 one row per thread,
 * 1 the row walk, 2 the block walk of a box (a band layout with offsets 1, nx,
 * nx ny, nx even and N even, whenever the row walk is chosen for it or the
 * block walk has at least 2048 workgroups: two x-adjacent rows per lane, two
 * lines by two planes per thread).  With 2 the
 * inner FP32 products of LF_PREC_MIXED take the block walk too when nx is a
 * multiple of 4 (four rows per lane), else the row walk; with 1 the row walk.
 * 3: DIC on the two-colour band layout with x-lines of a multiple of four
 * cells: the product, the sweeps, the DIC diagonal and the assembly with two
 * red-black pairs per lane (16-byte loads), under the same rule as the row
 * walk.
 * 4: form 2, and the FP64 solve with the diagonal preconditioner, where its
 * iteration's reductions are not folded into the update and direction (more
 * than 512 partials per slot), runs CG on the Jacobi-scaled system
 * S A S y = S b, S = diag(1/sqrt(diagB)) (unit diagonal; the same iterates as
 * the diagonally preconditioned CG of A in exact arithmetic, with the
 * residual norm still taken of b - A x): the iteration's product reads no
 * diagonal and its direction update no reciprocal, 16 bytes fewer per cell
 * and iteration; the scaled coefficients are formed once per solve.
 * lf_amul multiplies by A in every form.
 * All forms give bitwise the same product A x. */
lf_status lf_problem_amul_walk(const lf_problem *problem, int32_t *walk);

/* T[N]: on_device = 1 means a device pointer (copied on the handle's stream),
 * 0 a host pointer (synchronous).  lf_set_T rejects non-finite values. */
lf_status lf_set_T(lf_problem *problem, const double *T, int32_t on_device);
lf_status lf_get_T(lf_problem *problem, double *T, int32_t on_device);
/* Tb[B]: the field on the boundary faces, in boundary-face order (patch by
 * patch): the patch's value on fixedValue patches, the value of the face's cell
 * on zeroGradient patches (the boundary values that go with T; output only,
 * the solve does not use them).  on_device as for lf_get_T. */
lf_status lf_get_boundary_T(lf_problem *problem, double *Tb, int32_t on_device);

/* Gauss gradient of the problem's current T with its own boundary conditions
 * (Section 5.2, calcGrad of the solution field): lf_grad with T_b the values
 * of lf_get_boundary_T and snGrad_b = delta_b (T_b - T_P) on fixedValue patches,
 * 0 on zeroGradient ones.  grad[3N] and bgrad[3B] (may be NULL) are device
 * outputs, xyz interleaved, in the mesh's cell and boundary-face order, written
 * on the problem's stream (the call does not wait).  LF_EINVAL: NULL problem or
 * grad, or a mesh created without face centres; LF_ESTATE while an
 * lf_step_begin run is in flight. */
lf_status lf_problem_grad(lf_problem *problem, double *grad, double *bgrad);

/* Advance n_steps time steps.  stats[n_steps] (host, may be NULL).
 * Per step: assemble TEqn from the current T, solve from x0 = T, T = x.
 * Non-convergence is reported in stats, not as an error.  A non-finite
 * residual stops the call with LF_ENONFINITE after that step's stats. */
lf_status lf_step(lf_problem *problem, int32_t n_steps, lf_solve_stats *stats);

/* lf_step for n distinct problems at once: each advances n_steps time steps
 * exactly as lf_step would (same results), their device work interleaved so
 * that problems on different streams run concurrently; the host waits only
 * when every problem has work queued.  stats[n * n_steps] (host, problem-major,
 * may be NULL).  A problem whose step ends with a non-finite residual stops
 * there (its later stats are not written) while the others go on; the call
 * then returns LF_ENONFINITE.  For many medium-size problems whose single
 * solves cannot fill the GPU. */
lf_status lf_step_many(lf_problem *const *problems, int32_t n, int32_t n_steps, lf_solve_stats *stats);

/* lf_step without waiting: lf_step_begin enqueues the first of n_steps time
 * steps on the problem's stream and returns; lf_step_poll then advances the run
 * as far as its finished device work allows, without waiting for the device
 * (event queries only): it enqueues each next block of iterations or next step
 * and reports *steps_done and *finished (1 once all steps, or a step with a
 * non-finite residual, have finished; then LF_ENONFINITE is returned for the
 * latter).  Same results as lf_step.  snapshots (device, [n_steps][N] in the
 * mesh's cell order, may be NULL) receive T after each step, copied on the
 * problem's stream; stats[n_steps] (host, may be NULL) receives the stats of
 * the finished steps.  While a run is in flight the problem must not be
 * stepped, reset, assembled or read (lf_step, lf_step_many, lf_problem_reset,
 * lf_set_T, lf_get_T, lf_get_boundary_T, lf_problem_grad, lf_assemble,
 * lf_get_matrix, lf_amul and lf_batch_launch return LF_ESTATE); destroying it waits for
 * the run's device work.  For a scheduler that keeps several problems of
 * different sizes going without one waiting for another. */
lf_status lf_step_begin(lf_problem *problem, int32_t n_steps, double *snapshots);
lf_status lf_step_poll(lf_problem *problem, int32_t *steps_done, int32_t *finished, lf_solve_stats *stats);

/* ---- test hooks ------------------------------------------------------------ */
/* Assemble TEqn from the current T (no solve).  Then lf_get_matrix copies, to
 * host arrays (any may be NULL): diag[N] and source[N] of TEqn, upper[F],
 * diag_b[N] / source_b[N] (with the boundary internal / boundary coefficients
 * added, i.e. the matrix the solver sees), int_coeff[B], bou_coeff[B]. */
lf_status lf_assemble(lf_problem *problem);
lf_status lf_get_matrix(lf_problem *problem, double *diag, double *upper, double *source,
                        double *diag_b, double *source_b, double *int_coeff, double *bou_coeff);
/* y = A x with the last assembled solve-time matrix (diag_b, upper), in the
 * problem's layout and order of the solver's products; x, y device
 * pointers of N doubles, ordered on the handle's stream. */
lf_status lf_amul(lf_problem *problem, const double *x, double *y);
/* y = A32 x: the inner FP32 product of LF_PREC_MIXED with the FP32
 * coefficients the last step formed (the Jacobi-scaled matrix S A S, unit
 * diagonal), in the form the inner solve runs it (one row per thread, row
 * walk or block walk: bitwise the same).  x, y device pointers of N floats in
 * the solver's row order (the mesh's cell order unless lf_mesh_cell_order
 * reports a reordering), ordered on the handle's stream.  LF_EINVAL unless
 * LF_PREC_MIXED; LF_ESTATE before the first step (or after lf_problem_reset)
 * and during a run. */
lf_status lf_amul_inner(lf_problem *problem, const float *x, float *y);
/* w = M r: the FP64 solver's preconditioner (diagonal: w = (1/diag) r; DIC:
 * its diagonal from the last assembled matrix, then the forward and backward
 * sweeps; multigrid: the coarse matrices of the last assembled matrix, then
 * one cycle), as the solve applies it.  r, w device pointers of N doubles in
 * the mesh's cell order, ordered on the handle's stream; the problem's solver
 * vectors are overwritten (set T again before stepping).  LF_EINVAL for the
 * mixed-precision form; LF_ESTATE before lf_assemble or during a run. */
lf_status lf_precondition(lf_problem *problem, const double *r, double *w);

/* ---- batched form -------------------------------------------------------
 * Many independent problems (each its own mesh, boundary conditions, DT, dt
 * and T; created with LF_PREC_MIXED, the diagonal preconditioner and
 * LF_LAYOUT_ROWS; other problems give LF_EINVAL) advanced
 * by one persistent kernel: each workgroup takes the next problem of the task
 * table, in the order given, and runs all n_steps steps of it alone (assembly,
 * then the precision form's refinement with workgroup-level reductions).  A
 * problem's result does not depend on the other problems of the launch or on
 * n_workgroups; it depends on block_threads (the summation order inside the
 * workgroup).  Each step stops when the FP64 normalised residual is below a
 * tenth of tol (converged is reported against tol), like LF_PREC_MIXED.
 * The batch workspace holds the task table, a counter and the statistics. */
typedef struct lf_batch lf_batch;
size_t lf_batch_workspace_bytes(int32_t max_tasks, int32_t max_steps);
lf_status lf_batch_create(int32_t max_tasks, int32_t max_steps, void *dev_workspace,
                          size_t workspace_bytes, void *stream, lf_batch **out);
lf_status lf_batch_destroy(lf_batch *batch);     /* NULL-safe; waits for a launch in flight */
/* Enqueue on the batch's stream and return at once.  problems[n], n <= max_tasks,
 * n_steps <= max_steps, block_threads in {256, 512, 1024}, n_workgroups <= 0
 * means one per problem.  snapshots (may be NULL; entries may be NULL): for
 * problem i a device buffer of n_steps * N_i doubles that receives T after
 * each step, step-major.  The problems' T must be set (and any work on their
 * own streams finished) before the call; they must not be used until the
 * launch has finished (lf_batch_poll / lf_batch_wait).  LF_ESTATE if the
 * previous launch has not finished or a problem has an lf_step_begin run in
 * flight; LF_EINVAL if a problem is listed twice. */
lf_status lf_batch_launch(lf_batch *batch, int32_t n, lf_problem *const *problems,
                          double *const *snapshots, int32_t n_steps, int32_t block_threads,
                          int32_t n_workgroups);
lf_status lf_batch_poll(lf_batch *batch, int32_t *finished);   /* *finished = 1 when done */
lf_status lf_batch_wait(lf_batch *batch);
/* After the launch finished: stats[n * n_steps] (problem-major) and the device
 * time of the launch in milliseconds (either may be NULL). */
lf_status lf_batch_stats(lf_batch *batch, lf_solve_stats *stats, double *elapsed_ms);

/* ---- grouped form --------------------------------------------------------
 * Several LF_PREC_MIXED problems (diagonal preconditioner, orthogonal meshes,
 * FP64 products one row per thread: lf_problem_amul_walk reports 0) stepped
 * together, for many mid-size problems at once, each too small to fill the
 * GPU (the serving stream's large requests): every kernel of their steps runs
 * as one launch for all members that need it at that point (each member keeps
 * its own workgroups, rows and partial sums), on the group's stream.  Members join and
 * leave at any time: lf_group_add starts a member's run of n_steps steps,
 * lf_group_poll advances every member as far as finished device work allows
 * (event queries only; it never waits) and hands back the members whose runs
 * have finished.  A member's results (T after each step, stats) are bitwise
 * those of lf_step on the same problem, alone or with any other members.
 * Stats of a member report no times (assemble_ms = solve_ms = 0).  While a
 * member runs it must not be stepped, reset, read, set or destroyed (those
 * calls return LF_ESTATE).  The group workspace holds the members' descriptors
 * and their gathered solver states; the group's own launches go to `stream`. */
typedef struct lf_group lf_group;
size_t lf_group_workspace_bytes(int32_t max_members);   /* max_members <= 32 */
/* iters_per_block: inner iterations launched between two looks at the
 * members' states (0: 2; members whose pass ends inside a block idle through
 * the rest of it, so short blocks measured faster than long ones). */
lf_status lf_group_create(int32_t max_members, int32_t iters_per_block, void *dev_workspace,
                          size_t workspace_bytes, void *stream, lf_group **out);
/* LF_ESTATE if members are still running (the group is kept). */
lf_status lf_group_destroy(lf_group *group);    /* NULL-safe */
/* Start n_steps >= 1 steps of problem p from T0 (device, N doubles in the
 * mesh's cell order, copied by the group's next launch, after the work
 * already queued on the problem's stream; NULL: from its current T).  T0 is
 * not checked (a non-finite value ends the first step with a non-finite
 * residual).  T0, snapshots and stats must stay valid until the member is
 * handed back.  snapshots (device, [n_steps][N] in the mesh's cell order, may
 * be NULL) receive T after each step; stats (host, [n_steps], may be NULL)
 * receive each step's stats.
 * LF_EINVAL: a problem the group cannot run (see above) or on another device;
 * LF_ESTATE: the problem runs already (here, in another group or an
 * lf_step_begin run); LF_EBUDGET: the group is full. */
lf_status lf_group_add(lf_group *group, lf_problem *p, int32_t n_steps, const double *T0,
                       double *snapshots, lf_solve_stats *stats);
/* Advance; finished[0 .. *n_finished) receive the members whose runs finished
 * since the last call (at most max_finished; the rest on the next call) and
 * whose snapshots are complete; *n_active counts the members not yet handed
 * back.  A member whose step ended with a non-finite residual finishes there
 * (its stats say nonfinite).  LF_EDEVICE on a device error. */
lf_status lf_group_poll(lf_group *group, lf_problem **finished, int32_t max_finished, int32_t *n_finished,
                        int32_t *n_active);

/* ---- per-kernel device timing (diagnostics) ------------------------------
 * When enabled, lf_step records a HIP event pair around every kernel launch on
 * the handle's stream (plain launches instead of graphs, and a convergence
 * check after every iteration so that no launch is a no-op) and accumulates
 * the device time of each kernel class.  Each group of launches is preceded by
 * a 200 us GPU-side wait so the host has enqueued the group before the GPU
 * reaches it (the events then time the kernels, not the host); with timing on,
 * the stats' assemble_ms / solve_ms include those waits.  lf_profile_read copies, for class k in
 * [0, n_classes), the accumulated milliseconds to total_ms[k] and the launch
 * count to launches[k] (either may be NULL); lf_profile_enable(p, 1) also
 * clears the accumulators. */
#define LF_K_ASSEMBLE 0      /* cell-parallel TEqn assembly fused with A x0, r0,
                                normalisation terms and the first w.r */
#define LF_K_SETUP1 1        /* partial sums of x0 (mean for the normalisation) */
#define LF_K_COMMIT 2        /* last pending x += alpha p of a solve */
#define LF_K_DIRECTION 3     /* p = w + beta p, deferred x += alpha p */
#define LF_K_AMUL_DOT 4      /* q = A p, p.q partials */
#define LF_K_UPDATE 5        /* r -= alpha q, |r| and w.r partials */
#define LF_K_DIC_RD 6        /* DIC diagonal */
#define LF_K_DIC_FORWARD 7   /* DIC forward sweep (black rows) */
#define LF_K_DIC_BACKWARD 8  /* DIC backward sweep (red rows) + w.r partials */
#define LF_K_MIXED_RESIDUAL 9   /* mixed: FP64 residual r = b - A T, |r| partials */
#define LF_K_MIXED_CORRECT 10   /* mixed: T += d, FP32 copies */
#define LF_K_INNER_DIRECTION 11 /* mixed: FP32 direction update */
#define LF_K_INNER_AMUL_DOT 12  /* mixed: FP32 q = A p, FP64 p.q partials */
#define LF_K_INNER_UPDATE 13    /* mixed: FP32 update, FP64 partials */
#define LF_K_MIXED_PREP 14      /* mixed: FP32 coefficients of the scaled matrix
                                   (once per step) */
#define LF_K_FINALIZE 15        /* one-workgroup reductions and scalar decisions */
#define LF_K_AMG_SMOOTH 16      /* multigrid: Jacobi sweeps (all levels) */
#define LF_K_AMG_RESTRICT 17    /* multigrid: residual summed over the aggregates */
#define LF_K_AMG_PROLONG 18     /* multigrid: coarse correction added back */
#define LF_K_AMG_GALERKIN 19    /* multigrid: coarse matrices (once per step) */
#define LF_K_GRAD 20            /* non-orthogonal meshes: the gradient of T before
                                   each assembly (solver order) */
#define LF_K_NONORTH 21         /* non-orthogonal meshes without band form: the
                                   correction fluxes' divergence (band meshes form
                                   it inside the assembly) */
#define LF_K_SCALE 22           /* FP64 solves in product form 4: the coefficients
                                   of the Jacobi-scaled matrix (once per solve) */
#define LF_NUM_KERNEL_CLASSES 23
lf_status lf_profile_enable(lf_problem *problem, int32_t on);
lf_status lf_profile_read(lf_problem *problem, int32_t n_classes, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* LAPFOAM_H */
