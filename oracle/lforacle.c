/*
 * lforacle.c -- reference implementation (oracle) of one laplacianFoam time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library it checks.
 *
 * What it computes (Section 5.1, Eq. 1 and Listing 1 of the paper; readings of
 * what the paper leaves unstated are marked READING):
 *   one implicit-Euler step of  dT/dt - div(DT grad T) = 0  on a finite-volume
 *   mesh given in OpenFOAM face addressing (Section 4: owner / neighbour lists,
 *   face normal from owner to neighbour), assembled into an LDU matrix
 *   (diag, upper, lower = upper, source, per-boundary-face internal and
 *   boundary coefficients) and solved by the preconditioned conjugate gradient
 *   method with a diagonal or DIC preconditioner (Sections 5.1 and 6: PCG with
 *   the diagonal preconditioner);
 *   and the Gauss gradient of a cell field (Section 5.2: interpolation
 *   weights, face interpolation, gradf, division by the volume and the
 *   boundary correction), which the explicit non-orthogonal correction uses.
 *
 * Style: plain loops in the order the definitions state them, IEEE binary64,
 * compiled with -O2 -ffp-contract=off -fno-fast-math, single thread.  Every
 * sum runs sequentially in ascending index order.  No blocking, fusion or
 * reordering.
 *
 * Parity pins (checked by the CPU tests, not by this file): dense brute-force
 * stencil assembly on small boxes, numpy LU solve, 1-cell and 2-cell closed
 * forms, the exact steady linear profile, the exact discrete decay of a cosine
 * mode, the O(dx^2 + dt) decay of a sine mode, heat conservation, matrix
 * symmetry / row sums / diagonal dominance, and PCG special cases; for the
 * gradient: exactness for linear fields on skewed (affine) graded boxes,
 * central differences on uniform boxes, the discrete divergence identity
 * sum_c V_c g_c = sum_b S_b T_b, and the boundary correction's normal
 * component.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define LFO_OK 0
#define LFO_EINVAL (-1)
#define LFO_ENOMEM (-3)

#define BC_ZERO_GRADIENT 0
#define BC_FIXED_VALUE 1

#define PC_DIAGONAL 0
#define PC_DIC 1

typedef struct {
    double initial_residual;
    double final_residual;
    int32_t n_iter;
    int32_t converged;
    int32_t singular;
    int32_t pad;
    double assemble_s;
    double solve_s;
} lfo_stats;

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------------ */
/* Geometry (once per mesh).  READING: Gauss linear "corrected" Laplacian,   */
/* whose orthogonal part uses delta_f = 1/max(n.d, 0.05|d|) with n the unit  */
/* face normal and d = C_N - C_P; on boundary faces delta_b = 1/(n.(C_f-C_P)).*/
/* ------------------------------------------------------------------------ */
int lfo_face_geometry(int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
                      const double *cell_centre, const double *face_area,
                      double *mag_sf, double *delta)
{
    for (int32_t f = 0; f < n_faces; ++f) {
        const double *S = face_area + 3 * (size_t)f;
        double m = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
        double nx = S[0] / m, ny = S[1] / m, nz = S[2] / m;
        const double *P = cell_centre + 3 * (size_t)owner[f];
        const double *N = cell_centre + 3 * (size_t)neighbour[f];
        double dx = N[0] - P[0], dy = N[1] - P[1], dz = N[2] - P[2];
        double nd = nx * dx + ny * dy + nz * dz;
        double dmag = sqrt(dx * dx + dy * dy + dz * dz);
        double lim = 0.05 * dmag;
        mag_sf[f] = m;
        delta[f] = 1.0 / (nd > lim ? nd : lim);
    }
    return LFO_OK;
}

int lfo_bface_geometry(int32_t n_bfaces, const int32_t *bface_cell, const double *cell_centre,
                       const double *bface_area, const double *bface_centre,
                       double *bmag_sf, double *bdelta)
{
    for (int32_t b = 0; b < n_bfaces; ++b) {
        const double *S = bface_area + 3 * (size_t)b;
        double m = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
        double nx = S[0] / m, ny = S[1] / m, nz = S[2] / m;
        const double *P = cell_centre + 3 * (size_t)bface_cell[b];
        const double *F = bface_centre + 3 * (size_t)b;
        double dx = F[0] - P[0], dy = F[1] - P[1], dz = F[2] - P[2];
        double nd = nx * dx + ny * dy + nz * dz;
        bmag_sf[b] = m;
        bdelta[b] = 1.0 / nd;
    }
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Assembly of TEqn = ddt(T) - laplacian(DT, T)  (Listing 1).               */
/*  laplacian (Gauss): lapU_f = delta_f * (DT*|S_f|); lap diag by negated  */
/*   sum over the faces of each cell in face order; fixedValue boundary face */
/*   b: internalCoeff = -(DT|S_b|) delta_b, boundaryCoeff = -(DT|S_b|)       */
/*   (delta_b T_b); zeroGradient contributes nothing.                        */
/*  ddt (READING: implicit Euler): diag (1/dt) V, source ((1/dt) T_old) V.  */
/*  On a mesh with non-orthogonal faces the laplacian also has an explicit   */
/*  source lap_src (lfo_nonorth_source), which TEqn subtracts; NULL = none. */
/*  TEqn = ddt - laplacian, then the solve adds the boundary internal        */
/*  coefficients to diag and the boundary coefficients to source.            */
/* ------------------------------------------------------------------------ */
int lfo_assemble(int32_t n_cells, int32_t n_faces, const int32_t *owner,
                 const int32_t *neighbour, const double *cell_volume, const double *mag_sf,
                 const double *delta, int32_t n_patches, const int32_t *patch_start,
                 const int32_t *patch_type, const double *patch_value,
                 const int32_t *bface_cell, const double *bmag_sf, const double *bdelta,
                 double DT, double dt, const double *T_old, const double *lap_src,
                 double *diag, double *upper, double *source,
                 double *diag_b, double *source_b, double *int_coeff, double *bou_coeff)
{
    if (n_cells < 0 || n_faces < 0 || !(dt > 0.0))
        return LFO_EINVAL;
    double *lap_diag = (double *)malloc(sizeof(double) * (size_t)(n_cells > 0 ? n_cells : 1));
    if (!lap_diag)
        return LFO_ENOMEM;

    /* laplacian: upper and negSumDiag */
    for (int32_t c = 0; c < n_cells; ++c)
        lap_diag[c] = 0.0;
    for (int32_t f = 0; f < n_faces; ++f) {
        double gamma_mag_sf = DT * mag_sf[f];
        double lap_upper = delta[f] * gamma_mag_sf;
        upper[f] = -lap_upper; /* TEqn upper = 0 - laplacian upper */
        lap_diag[owner[f]] -= lap_upper; /* lower = upper (symmetric) */
        lap_diag[neighbour[f]] -= lap_upper;
    }

    /* ddt (Euler) minus laplacian */
    double rdt = 1.0 / dt;
    for (int32_t c = 0; c < n_cells; ++c) {
        double ddt_diag = rdt * cell_volume[c];
        diag[c] = ddt_diag - lap_diag[c];
        source[c] = (rdt * T_old[c]) * cell_volume[c];
        if (lap_src) /* the laplacian's explicit non-orthogonal source, subtracted */
            source[c] = source[c] - lap_src[c];
    }
    free(lap_diag);

    /* boundary coefficients of TEqn (= 0 - laplacian's) */
    for (int32_t p = 0; p < n_patches; ++p) {
        for (int32_t b = patch_start[p]; b < patch_start[p + 1]; ++b) {
            if (patch_type[p] == BC_FIXED_VALUE) {
                double gamma_b = DT * bmag_sf[b];
                double lap_ic = gamma_b * (-bdelta[b]);
                double lap_bc = -(gamma_b * (bdelta[b] * patch_value[p]));
                int_coeff[b] = 0.0 - lap_ic;
                bou_coeff[b] = 0.0 - lap_bc;
            } else {
                int_coeff[b] = 0.0;
                bou_coeff[b] = 0.0;
            }
        }
    }

    /* solve-time matrix: add boundary diag and source, patch order, face order */
    for (int32_t c = 0; c < n_cells; ++c) {
        diag_b[c] = diag[c];
        source_b[c] = source[c];
    }
    for (int32_t p = 0; p < n_patches; ++p) {
        if (patch_type[p] != BC_FIXED_VALUE)
            continue;
        for (int32_t b = patch_start[p]; b < patch_start[p + 1]; ++b) {
            diag_b[bface_cell[b]] += int_coeff[b];
            source_b[bface_cell[b]] += bou_coeff[b];
        }
    }
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* LDU matrix-vector product: y = A x, diag first, then faces ascending.    */
/* ------------------------------------------------------------------------ */
int lfo_amul(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
             const double *diag, const double *upper, const double *x, double *y)
{
    for (int32_t c = 0; c < n_cells; ++c)
        y[c] = diag[c] * x[c];
    for (int32_t f = 0; f < n_faces; ++f) {
        y[neighbour[f]] += upper[f] * x[owner[f]]; /* lower = upper */
        y[owner[f]] += upper[f] * x[neighbour[f]];
    }
    return LFO_OK;
}

/* row sums of A: diag plus the off-diagonal coefficients of each row */
int lfo_sum_a(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
              const double *diag, const double *upper, double *sum_a)
{
    for (int32_t c = 0; c < n_cells; ++c)
        sum_a[c] = diag[c];
    for (int32_t f = 0; f < n_faces; ++f) {
        sum_a[owner[f]] += upper[f]; /* lower coefficient of row owner */
        sum_a[neighbour[f]] += upper[f];
    }
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Preconditioners.                                                          */
/*  diagonal: rD = 1/diag, w = rD r.                                         */
/*  DIC (READING: the classic diagonal incomplete Cholesky, Barrett et al.   */
/*  "Templates", 1994): rD_c = diag_c - sum over lower faces (upper^2)/rD_l, */
/*  in face order, then rD = 1/rD; apply w = rD r, a forward sweep           */
/*  w_u -= rD_u upper w_l (faces ascending), a backward sweep                */
/*  w_l -= rD_l upper w_u (faces descending).                                */
/* ------------------------------------------------------------------------ */
int lfo_dic_rd(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
               const double *diag, const double *upper, double *rd)
{
    for (int32_t c = 0; c < n_cells; ++c)
        rd[c] = diag[c];
    for (int32_t f = 0; f < n_faces; ++f)
        rd[neighbour[f]] -= upper[f] * upper[f] / rd[owner[f]];
    for (int32_t c = 0; c < n_cells; ++c)
        rd[c] = 1.0 / rd[c];
    return LFO_OK;
}

static void precondition(int pc, int32_t n_cells, int32_t n_faces, const int32_t *owner,
                         const int32_t *neighbour, const double *upper, const double *rd,
                         const double *r, double *w)
{
    for (int32_t c = 0; c < n_cells; ++c)
        w[c] = rd[c] * r[c];
    if (pc != PC_DIC)
        return;
    for (int32_t f = 0; f < n_faces; ++f)
        w[neighbour[f]] -= rd[neighbour[f]] * upper[f] * w[owner[f]];
    for (int32_t f = n_faces - 1; f >= 0; --f)
        w[owner[f]] -= rd[owner[f]] * upper[f] * w[neighbour[f]];
}

int lfo_precondition(int pc, int32_t n_cells, int32_t n_faces, const int32_t *owner,
                     const int32_t *neighbour, const double *upper, const double *rd,
                     const double *r, double *w)
{
    precondition(pc, n_cells, n_faces, owner, neighbour, upper, rd, r, w);
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Aggregation multigrid preconditioner (Section 7 names an algebraic       */
/* multigrid library as the better alternative to the diagonal PCG).        */
/* READING (the paper gives no cycle): a V-cycle over Galerkin coarse       */
/* matrices A_{l+1} = P^T A_l P, with P the piecewise-constant prolongation */
/* of an aggregation of the cells (agg_l[c] = the coarse cell holding c):   */
/*   coarse diag_I = sum over the cells of I (ascending) of diag_c, then    */
/*     plus 2 upper_f for each face inside I (ascending face order);        */
/*   coarse upper of the pair (I, J), I < J = the sum over the faces        */
/*     joining I and J (ascending face order), pairs in upper-triangular    */
/*     order.                                                               */
/* Smoother: weighted Jacobi, x_c = x_c + omega ((b_c - (A x)_c) / diag_c). */
/* Cycle on level l for b: x = 0; nu sweeps; r = b - A x; the coarse right  */
/* side sums r over each aggregate (ascending cells); cycle on level l + 1; */
/* x_c += coarse x of c's aggregate; nu sweeps.  On the coarsest level:     */
/* nu_c sweeps from x = 0.  With the same sweeps before and after, the      */
/* cycle is a symmetric operator, as PCG needs.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n, nf;
    const int32_t *owner, *neighbour;
    const double *diag, *upper;
    const int32_t *agg;      /* [n] coarse cell of each cell; NULL on the coarsest level */
} amg_level;

typedef struct {
    int32_t n_levels, nu, nu_c;
    double omega;
    amg_level *lv;           /* levels 1.. own their arrays */
} amg_hier;

typedef struct {
    int32_t I, J, f;
} amg_pair;

static int cmp_amg_pair(const void *a, const void *b)
{
    const amg_pair *p = (const amg_pair *)a, *q = (const amg_pair *)b;
    if (p->I != q->I)
        return p->I < q->I ? -1 : 1;
    if (p->J != q->J)
        return p->J < q->J ? -1 : 1;
    return p->f < q->f ? -1 : (p->f > q->f);
}

/* Galerkin coarse matrix of (fine matrix, aggregation into nc cells).  The
 * coarse face arrays must hold up to nf entries; *nfc receives their count. */
int lfo_galerkin(int32_t n, int32_t nf, const int32_t *owner, const int32_t *neighbour,
                 const double *diag, const double *upper, const int32_t *agg, int32_t nc,
                 int32_t *nfc, int32_t *cowner, int32_t *cneighbour, double *cdiag, double *cupper)
{
    if (n < 1 || nf < 0 || nc < 1)
        return LFO_EINVAL;
    for (int32_t c = 0; c < n; ++c)
        if (agg[c] < 0 || agg[c] >= nc)
            return LFO_EINVAL;
    amg_pair *pairs = (amg_pair *)malloc(sizeof(amg_pair) * (size_t)(nf > 0 ? nf : 1));
    if (!pairs)
        return LFO_ENOMEM;
    for (int32_t I = 0; I < nc; ++I)
        cdiag[I] = 0.0;
    for (int32_t c = 0; c < n; ++c)
        cdiag[agg[c]] += diag[c];
    int32_t m = 0;
    for (int32_t f = 0; f < nf; ++f) {
        int32_t I = agg[owner[f]], J = agg[neighbour[f]];
        if (I == J) {
            cdiag[I] += 2.0 * upper[f];
        } else {
            pairs[m].I = I < J ? I : J;
            pairs[m].J = I < J ? J : I;
            pairs[m].f = f;
            ++m;
        }
    }
    qsort(pairs, (size_t)m, sizeof(amg_pair), cmp_amg_pair);
    int32_t k = -1;
    for (int32_t i = 0; i < m; ++i) {
        if (i == 0 || pairs[i].I != pairs[i - 1].I || pairs[i].J != pairs[i - 1].J) {
            ++k;
            cowner[k] = pairs[i].I;
            cneighbour[k] = pairs[i].J;
            cupper[k] = 0.0;
        }
        cupper[k] += upper[pairs[i].f];
    }
    *nfc = k + 1;
    free(pairs);
    return LFO_OK;
}

static void amg_free(amg_hier *h)
{
    if (!h->lv)
        return;
    for (int32_t l = 1; l < h->n_levels; ++l) {
        free((void *)h->lv[l].owner);
        free((void *)h->lv[l].neighbour);
        free((void *)h->lv[l].diag);
        free((void *)h->lv[l].upper);
    }
    free(h->lv);
    h->lv = NULL;
}

/* level_cells[n_levels]: cells per level (level_cells[0] = n); aggs: the
 * aggregation of each level but the last, concatenated. */
static int amg_build(int32_t n, int32_t nf, const int32_t *owner, const int32_t *neighbour,
                     const double *diag, const double *upper, int32_t n_levels,
                     const int32_t *level_cells, const int32_t *aggs, int32_t nu, int32_t nu_c,
                     double omega, amg_hier *h)
{
    h->lv = NULL;
    if (n_levels < 1 || level_cells[0] != n || nu < 0 || nu_c < 0)
        return LFO_EINVAL;
    h->n_levels = n_levels;
    h->nu = nu;
    h->nu_c = nu_c;
    h->omega = omega;
    h->lv = (amg_level *)calloc((size_t)n_levels, sizeof(amg_level));
    if (!h->lv)
        return LFO_ENOMEM;
    h->lv[0].n = n;
    h->lv[0].nf = nf;
    h->lv[0].owner = owner;
    h->lv[0].neighbour = neighbour;
    h->lv[0].diag = diag;
    h->lv[0].upper = upper;
    const int32_t *a = aggs;
    for (int32_t l = 0; l + 1 < n_levels; ++l) {
        amg_level *F = &h->lv[l], *C = &h->lv[l + 1];
        F->agg = a;
        a += F->n;
        int32_t nc = level_cells[l + 1];
        size_t cap = (size_t)(F->nf > 0 ? F->nf : 1);
        int32_t *co = (int32_t *)malloc(sizeof(int32_t) * cap);
        int32_t *cn = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *cd = (double *)malloc(sizeof(double) * (size_t)nc);
        double *cu = (double *)malloc(sizeof(double) * cap);
        C->owner = co;
        C->neighbour = cn;
        C->diag = cd;
        C->upper = cu;
        C->n = nc;
        if (!co || !cn || !cd || !cu) {
            h->n_levels = l + 2;
            amg_free(h);
            return LFO_ENOMEM;
        }
        int rc = lfo_galerkin(F->n, F->nf, F->owner, F->neighbour, F->diag, F->upper, F->agg, nc,
                              &C->nf, co, cn, cd, cu);
        if (rc != LFO_OK) {
            h->n_levels = l + 2;
            amg_free(h);
            return rc;
        }
    }
    return LFO_OK;
}

static void amg_jacobi(const amg_level *L, double omega, const double *b, double *x, double *y)
{
    lfo_amul(L->n, L->nf, L->owner, L->neighbour, L->diag, L->upper, x, y);
    for (int32_t c = 0; c < L->n; ++c)
        x[c] = x[c] + omega * ((b[c] - y[c]) / L->diag[c]);
}

static int amg_vcycle(const amg_hier *h, int32_t l, const double *b, double *x)
{
    const amg_level *L = &h->lv[l];
    double *y = (double *)malloc(sizeof(double) * (size_t)L->n);
    if (!y)
        return LFO_ENOMEM;
    for (int32_t c = 0; c < L->n; ++c)
        x[c] = 0.0;
    if (l == h->n_levels - 1) {
        for (int32_t s = 0; s < h->nu_c; ++s)
            amg_jacobi(L, h->omega, b, x, y);
        free(y);
        return LFO_OK;
    }
    for (int32_t s = 0; s < h->nu; ++s)
        amg_jacobi(L, h->omega, b, x, y);
    lfo_amul(L->n, L->nf, L->owner, L->neighbour, L->diag, L->upper, x, y);
    for (int32_t c = 0; c < L->n; ++c)
        y[c] = b[c] - y[c];
    const amg_level *C = &h->lv[l + 1];
    double *bc = (double *)calloc((size_t)C->n, sizeof(double));
    double *xc = (double *)malloc(sizeof(double) * (size_t)C->n);
    if (!bc || !xc) {
        free(y); free(bc); free(xc);
        return LFO_ENOMEM;
    }
    for (int32_t c = 0; c < L->n; ++c)
        bc[L->agg[c]] += y[c];
    int rc = amg_vcycle(h, l + 1, bc, xc);
    if (rc == LFO_OK) {
        for (int32_t c = 0; c < L->n; ++c)
            x[c] += xc[L->agg[c]];
        for (int32_t s = 0; s < h->nu; ++s)
            amg_jacobi(L, h->omega, b, x, y);
    }
    free(y); free(bc); free(xc);
    return rc;
}

/* One application of the cycle: w = M r. */
int lfo_amg_apply(int32_t n, int32_t nf, const int32_t *owner, const int32_t *neighbour,
                  const double *diag, const double *upper, int32_t n_levels,
                  const int32_t *level_cells, const int32_t *aggs, int32_t nu, int32_t nu_c,
                  double omega, const double *r, double *w)
{
    amg_hier h;
    int rc = amg_build(n, nf, owner, neighbour, diag, upper, n_levels, level_cells, aggs, nu, nu_c,
                       omega, &h);
    if (rc == LFO_OK)
        rc = amg_vcycle(&h, 0, r, w);
    amg_free(&h);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* PCG (READING: OpenFOAM's PCG semantics).                                  */
/*  r = b - A x0;  normFactor = sum_c(|Ax0_c - pA_c| + |b_c - pA_c|) + 1e-20 */
/*  with pA = (row sums of A) * mean(x0);  res = sum|r| / normFactor.        */
/*  Converged iff res < tol or (relTol > 1e-20 and res < relTol res0).       */
/*  Checked before the loop and after each iteration (the check after an     */
/*  iteration is skipped once maxIter is reached).  Singular iff             */
/*  |wApA|/normFactor < 1e-300, which ends the loop without counting the     */
/*  iteration.                                                                */
/* ------------------------------------------------------------------------ */
static int check_conv(double res, double res0, double tol, double rel_tol)
{
    return (res < tol) || (rel_tol > 1e-20 && res < rel_tol * res0);
}

/* The loop below with the preconditioner pc, or with the cycle of amg when
 * amg is not NULL. */
static int pcg_core(int32_t n_cells, int32_t n_faces, const int32_t *owner,
                    const int32_t *neighbour, const double *diag, const double *upper,
                    const double *b, double *x, int pc, const amg_hier *amg, double tol,
                    double rel_tol, int32_t max_iter, int32_t min_iter, lfo_stats *st)
{
    size_t n = (size_t)(n_cells > 0 ? n_cells : 1);
    double *wA = (double *)malloc(sizeof(double) * n);
    double *rA = (double *)malloc(sizeof(double) * n);
    double *pA = (double *)malloc(sizeof(double) * n);
    double *rD = (double *)malloc(sizeof(double) * n);
    if (!wA || !rA || !pA || !rD) {
        free(wA); free(rA); free(pA); free(rD);
        return LFO_ENOMEM;
    }
    st->n_iter = 0;
    st->converged = 0;
    st->singular = 0;

    lfo_amul(n_cells, n_faces, owner, neighbour, diag, upper, x, wA);
    for (int32_t c = 0; c < n_cells; ++c)
        rA[c] = b[c] - wA[c];

    /* normalisation factor */
    lfo_sum_a(n_cells, n_faces, owner, neighbour, diag, upper, pA);
    double sum_x = 0.0;
    for (int32_t c = 0; c < n_cells; ++c)
        sum_x += x[c];
    double x_avg = sum_x / (double)n_cells;
    for (int32_t c = 0; c < n_cells; ++c)
        pA[c] *= x_avg;
    double norm_factor = 0.0;
    for (int32_t c = 0; c < n_cells; ++c)
        norm_factor += fabs(wA[c] - pA[c]) + fabs(b[c] - pA[c]);
    norm_factor += 1e-20;

    double sum_mag = 0.0;
    for (int32_t c = 0; c < n_cells; ++c)
        sum_mag += fabs(rA[c]);
    st->initial_residual = sum_mag / norm_factor;
    st->final_residual = st->initial_residual;
    st->converged = check_conv(st->final_residual, st->initial_residual, tol, rel_tol);

    if (min_iter > 0 || !st->converged) {
        if (pc == PC_DIC) {
            lfo_dic_rd(n_cells, n_faces, owner, neighbour, diag, upper, rD);
        } else {
            for (int32_t c = 0; c < n_cells; ++c)
                rD[c] = 1.0 / diag[c];
        }
        double wArA = 1e20, wArA_old;
        for (;;) {
            wArA_old = wArA;
            if (amg) {
                int rc = amg_vcycle(amg, 0, rA, wA);
                if (rc != LFO_OK) {
                    free(wA); free(rA); free(pA); free(rD);
                    return rc;
                }
            } else {
                precondition(pc, n_cells, n_faces, owner, neighbour, upper, rD, rA, wA);
            }
            wArA = 0.0;
            for (int32_t c = 0; c < n_cells; ++c)
                wArA += wA[c] * rA[c];
            if (st->n_iter == 0) {
                for (int32_t c = 0; c < n_cells; ++c)
                    pA[c] = wA[c];
            } else {
                double beta = wArA / wArA_old;
                for (int32_t c = 0; c < n_cells; ++c)
                    pA[c] = wA[c] + beta * pA[c];
            }
            lfo_amul(n_cells, n_faces, owner, neighbour, diag, upper, pA, wA);
            double wApA = 0.0;
            for (int32_t c = 0; c < n_cells; ++c)
                wApA += wA[c] * pA[c];
            if (fabs(wApA) / norm_factor < 1e-300) {
                st->singular = 1;
                break;
            }
            double alpha = wArA / wApA;
            for (int32_t c = 0; c < n_cells; ++c) {
                x[c] += alpha * pA[c];
                rA[c] -= alpha * wA[c];
            }
            sum_mag = 0.0;
            for (int32_t c = 0; c < n_cells; ++c)
                sum_mag += fabs(rA[c]);
            st->final_residual = sum_mag / norm_factor;
            ++st->n_iter;
            if (st->n_iter < max_iter)
                st->converged = check_conv(st->final_residual, st->initial_residual, tol,
                                           rel_tol);
            if (!((st->n_iter < max_iter && !st->converged) || st->n_iter < min_iter))
                break;
        }
    }
    free(wA); free(rA); free(pA); free(rD);
    return LFO_OK;
}

int lfo_pcg(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
            const double *diag, const double *upper, const double *b, double *x,
            int pc, double tol, double rel_tol, int32_t max_iter, int32_t min_iter,
            lfo_stats *st)
{
    return pcg_core(n_cells, n_faces, owner, neighbour, diag, upper, b, x, pc, NULL, tol, rel_tol,
                    max_iter, min_iter, st);
}

/* PCG preconditioned by the aggregation multigrid cycle above. */
int lfo_pcg_amg(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
                const double *diag, const double *upper, const double *b, double *x,
                int32_t n_levels, const int32_t *level_cells, const int32_t *aggs, int32_t nu,
                int32_t nu_c, double omega, double tol, double rel_tol, int32_t max_iter,
                int32_t min_iter, lfo_stats *st)
{
    amg_hier h;
    int rc = amg_build(n_cells, n_faces, owner, neighbour, diag, upper, n_levels, level_cells, aggs,
                       nu, nu_c, omega, &h);
    if (rc == LFO_OK)
        rc = pcg_core(n_cells, n_faces, owner, neighbour, diag, upper, b, x, PC_DIAGONAL, &h, tol,
                      rel_tol, max_iter, min_iter, st);
    amg_free(&h);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Time loop (Listing 1 with one non-orthogonal pass and empty fvOptions):  */
/* per step assemble, solve from x0 = T_old, commit T_new = x.              */
/* ------------------------------------------------------------------------ */
int lfo_run(int32_t n_cells, int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
            const double *cell_volume, const double *cell_centre, const double *face_area,
            int32_t n_patches, const int32_t *patch_start, const int32_t *patch_type,
            const double *patch_value, const int32_t *bface_cell, const double *bface_area,
            const double *bface_centre, double DT, double dt, int32_t n_steps, int pc,
            double tol, double rel_tol, int32_t max_iter, int32_t min_iter,
            double *T, lfo_stats *stats)
{
    if (n_cells <= 0 || n_faces < 0 || n_patches < 0 || n_steps < 0 || !(dt > 0.0))
        return LFO_EINVAL;
    int32_t n_b = patch_start[n_patches];
    size_t nc = (size_t)n_cells, nf = (size_t)(n_faces > 0 ? n_faces : 1);
    size_t nb = (size_t)(n_b > 0 ? n_b : 1);
    double *mag_sf = (double *)malloc(sizeof(double) * nf);
    double *delta = (double *)malloc(sizeof(double) * nf);
    double *bmag_sf = (double *)malloc(sizeof(double) * nb);
    double *bdelta = (double *)malloc(sizeof(double) * nb);
    double *diag = (double *)malloc(sizeof(double) * nc);
    double *upper = (double *)malloc(sizeof(double) * nf);
    double *source = (double *)malloc(sizeof(double) * nc);
    double *diag_b = (double *)malloc(sizeof(double) * nc);
    double *source_b = (double *)malloc(sizeof(double) * nc);
    double *ic = (double *)malloc(sizeof(double) * nb);
    double *bc = (double *)malloc(sizeof(double) * nb);
    int rc = LFO_OK;
    if (!mag_sf || !delta || !bmag_sf || !bdelta || !diag || !upper || !source || !diag_b ||
        !source_b || !ic || !bc) {
        rc = LFO_ENOMEM;
        goto done;
    }
    lfo_face_geometry(n_faces, owner, neighbour, cell_centre, face_area, mag_sf, delta);
    lfo_bface_geometry(n_b, bface_cell, cell_centre, bface_area, bface_centre, bmag_sf, bdelta);
    for (int32_t s = 0; s < n_steps; ++s) {
        double t0 = now_s();
        rc = lfo_assemble(n_cells, n_faces, owner, neighbour, cell_volume, mag_sf, delta,
                          n_patches, patch_start, patch_type, patch_value, bface_cell, bmag_sf,
                          bdelta, DT, dt, T, NULL, diag, upper, source, diag_b, source_b, ic, bc);
        if (rc != LFO_OK)
            goto done;
        double t1 = now_s();
        rc = lfo_pcg(n_cells, n_faces, owner, neighbour, diag_b, upper, source_b, T, pc, tol,
                     rel_tol, max_iter, min_iter, &stats[s]);
        if (rc != LFO_OK)
            goto done;
        double t2 = now_s();
        stats[s].assemble_s = t1 - t0;
        stats[s].solve_s = t2 - t1;
    }
done:
    free(mag_sf); free(delta); free(bmag_sf); free(bdelta); free(diag); free(upper);
    free(source); free(diag_b); free(source_b); free(ic); free(bc);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Gauss gradient of a cell field (Section 5.2, "calcGrad": interpolation, */
/* then gradf, then correctBoundaryConditions).  Not part of the time step  */
/* on orthogonal meshes: it feeds the explicit non-orthogonal correction.   */
/* ------------------------------------------------------------------------ */

/* Linear interpolation weights (Section 5.2, the weights loop): with the two
 * projected distances SfdOwn = |S_f.(C_f - C_P)| and SfdNei = |S_f.(C_N - C_f)|
 * the owner's weight is w_f = SfdNei / (SfdOwn + SfdNei), the neighbour-side
 * share, so that a field linear along the line P-N is reproduced at the face;
 * when |SfdOwn + SfdNei| is not above ROOTVSMALL the weight is 1/2.
 * READING: the paper names ROOTVSMALL without its value; OpenFOAM's
 * double-precision value is the square root of VSMALL = 1e-300, i.e. 1e-150. */
#define LFO_ROOTVSMALL 1.0e-150
int lfo_interp_weights(int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
                       const double *cell_centre, const double *face_area,
                       const double *face_centre, double *w)
{
    for (int32_t f = 0; f < n_faces; ++f) {
        const double *S = face_area + 3 * (size_t)f;
        const double *Cf = face_centre + 3 * (size_t)f;
        const double *P = cell_centre + 3 * (size_t)owner[f];
        const double *N = cell_centre + 3 * (size_t)neighbour[f];
        double sfd_own = fabs(S[0] * (Cf[0] - P[0]) + S[1] * (Cf[1] - P[1]) + S[2] * (Cf[2] - P[2]));
        double sfd_nei = fabs(S[0] * (N[0] - Cf[0]) + S[1] * (N[1] - Cf[1]) + S[2] * (N[2] - Cf[2]));
        double den = sfd_own + sfd_nei;
        w[f] = fabs(den) > LFO_ROOTVSMALL ? sfd_nei / den : 0.5;
    }
    return LFO_OK;
}

/* Face values of a cell field (Section 5.2, the interpolation loop):
 * s_f = w_f (v_P - v_N) + v_N. */
int lfo_interpolate(int32_t n_faces, const int32_t *owner, const int32_t *neighbour,
                    const double *w, const double *v, double *s)
{
    for (int32_t f = 0; f < n_faces; ++f)
        s[f] = w[f] * (v[owner[f]] - v[neighbour[f]]) + v[neighbour[f]];
    return LFO_OK;
}

/* Boundary values of T and their normal gradient for the two conditions of
 * the solver.  READING (the paper uses the boundary field without stating
 * it): fixedValue T_b = value, snGrad_b = delta_b (T_b - T_P); zeroGradient
 * T_b = T_P, snGrad_b = 0. */
int lfo_boundary_values(int32_t n_patches, const int32_t *patch_start, const int32_t *patch_type,
                        const double *patch_value, const int32_t *bface_cell, const double *bdelta,
                        const double *T, double *Tb, double *snb)
{
    for (int32_t p = 0; p < n_patches; ++p) {
        for (int32_t b = patch_start[p]; b < patch_start[p + 1]; ++b) {
            double Tc = T[bface_cell[b]];
            if (patch_type[p] == BC_FIXED_VALUE) {
                Tb[b] = patch_value[p];
                snb[b] = bdelta[b] * (patch_value[p] - Tc);
            } else if (patch_type[p] == BC_ZERO_GRADIENT) {
                Tb[b] = Tc;
                snb[b] = 0.0;
            } else {
                return LFO_EINVAL;
            }
        }
    }
    return LFO_OK;
}

/* gradf and correctBoundaryConditions (Section 5.2):
 *  g_c = 0; for each internal face in face order: g_P += S_f s_f,
 *  g_N -= S_f s_f; for each boundary face in order: g_c += S_b T_b;
 *  then g_c /= V_c.
 *  Boundary value of the gradient: the face cell's gradient, corrected to
 *  the boundary's normal gradient, g_b = g_P + n (snGrad_b - n.g_P) with
 *  n = S_b / |S_b|.
 * grad[3N] and bgrad[3B] are xyz interleaved. */
int lfo_gauss_grad(int32_t n_cells, int32_t n_faces, const int32_t *owner,
                   const int32_t *neighbour, const double *cell_volume, const double *face_area,
                   const double *s, int32_t n_bfaces, const int32_t *bface_cell,
                   const double *bface_area, const double *Tb, const double *snb,
                   double *grad, double *bgrad)
{
    for (int64_t i = 0; i < 3 * (int64_t)n_cells; ++i)
        grad[i] = 0.0;
    for (int32_t f = 0; f < n_faces; ++f) {
        const double *S = face_area + 3 * (size_t)f;
        double *gP = grad + 3 * (size_t)owner[f];
        double *gN = grad + 3 * (size_t)neighbour[f];
        for (int k = 0; k < 3; ++k) {
            double v = S[k] * s[f];
            gP[k] += v;
            gN[k] -= v;
        }
    }
    for (int32_t b = 0; b < n_bfaces; ++b) {
        const double *S = bface_area + 3 * (size_t)b;
        double *g = grad + 3 * (size_t)bface_cell[b];
        for (int k = 0; k < 3; ++k)
            g[k] += S[k] * Tb[b];
    }
    for (int32_t c = 0; c < n_cells; ++c)
        for (int k = 0; k < 3; ++k)
            grad[3 * (size_t)c + k] /= cell_volume[c];
    for (int32_t b = 0; b < n_bfaces; ++b) {
        const double *S = bface_area + 3 * (size_t)b;
        const double *g = grad + 3 * (size_t)bface_cell[b];
        double m = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
        double n[3] = {S[0] / m, S[1] / m, S[2] / m};
        double ng = n[0] * g[0] + n[1] * g[1] + n[2] * g[2];
        double d = snb[b] - ng;
        for (int k = 0; k < 3; ++k)
            bgrad[3 * (size_t)b + k] = g[k] + n[k] * d;
    }
    return LFO_OK;
}

/* ------------------------------------------------------------------------ */
/* Explicit non-orthogonal correction of the Gauss linear corrected         */
/* Laplacian (Section 5.1: the loop of non-orthogonal correctors around     */
/* TEqn, whose explicit part is what the gradient of Section 5.2 feeds).     */
/* READING (the scheme's standard form; the paper names it without          */
/* stating it): the face's correction vector k_f = n_f - delta_f d_f        */
/* (n_f = S_f/|S_f|, d_f = C_N - C_P, delta_f as for the implicit part),     */
/* the face gradient interpolated linearly g_f = w_f (g_P - g_N) + g_N per   */
/* component, the face flux (DT |S_f|) (k_f . g_f), its divergence          */
/* div_c = (sum over owned faces - sum over neighbour faces) / V_c (no       */
/* boundary face contributes: k_b = 0 on non-coupled patches), and the      */
/* laplacian's source lap_src_c = 0 - V_c div_c.  With one pass of the      */
/* corrector loop (no extra correctors) g is the gradient of T at assembly. */
/* ------------------------------------------------------------------------ */
int lfo_nonorth_source(int32_t n_cells, int32_t n_faces, const int32_t *owner,
                       const int32_t *neighbour, const double *cell_volume,
                       const double *cell_centre, const double *face_area, const double *mag_sf,
                       const double *delta, const double *w, const double *grad, double DT,
                       double *lap_src)
{
    double *div = (double *)malloc(sizeof(double) * (size_t)(n_cells > 0 ? n_cells : 1));
    if (!div)
        return LFO_ENOMEM;
    for (int32_t c = 0; c < n_cells; ++c)
        div[c] = 0.0;
    for (int32_t f = 0; f < n_faces; ++f) {
        const double *S = face_area + 3 * (size_t)f;
        const double *P = cell_centre + 3 * (size_t)owner[f];
        const double *N = cell_centre + 3 * (size_t)neighbour[f];
        const double *gP = grad + 3 * (size_t)owner[f];
        const double *gN = grad + 3 * (size_t)neighbour[f];
        double k[3], gf[3];
        for (int i = 0; i < 3; ++i) {
            k[i] = S[i] / mag_sf[f] - delta[f] * (N[i] - P[i]);
            gf[i] = w[f] * (gP[i] - gN[i]) + gN[i];
        }
        double corr = k[0] * gf[0] + k[1] * gf[1] + k[2] * gf[2];
        double flux = (DT * mag_sf[f]) * corr;
        div[owner[f]] += flux;
        div[neighbour[f]] -= flux;
    }
    for (int32_t c = 0; c < n_cells; ++c) {
        div[c] /= cell_volume[c];
        lap_src[c] = 0.0 - cell_volume[c] * div[c];
    }
    free(div);
    return LFO_OK;
}
