// Gauss gradient of a cell field (Section 5.2: calcGrad = interpolate, gradf,
// correctBoundaryConditions), gathered per cell: over the row layout built
// from the lists of lists, or, on meshes with band form, from band slots.
//
// The paper parallelises the face loop of gradf, which scatters S_f s_f to the
// owner (+) and the neighbour (-) of each face, by turning it into a gather:
// each cell walks its faces through ownerStart/ownerList and
// neighbourStart/neighbourList, then its boundary faces through
// facePatchStart.  Here one thread does that for one cell, with the face
// interpolation s_f = w_f (T_P - T_N) + T_N fused in (recomputed on each side
// of the face, the same value both times) and the division by V_c and the
// boundary correction of the cell's boundary faces fused after it, so a cell's
// gradient costs one launch and no face-sized intermediate.
//
// Order of the sums: the sequential loop reaches cell c first through the
// faces whose neighbour is c (their owners are smaller, so those faces come
// earlier in upper-triangular order), in ascending face order, then through
// the faces c owns, ascending, then through its boundary faces, ascending.
// The gather takes the same order and the library is built without
// multiply-add contraction, so every result equals the sequential loop's bit
// for bit.
//
// Face records: {S_x, S_y, S_z, w_f} per internal face and {S_x, S_y, S_z,
// |S_b|} per boundary face, 32 bytes each, read as two 16-byte loads.
#include <mutex>

#include "lf_solver.h"

namespace lf {

// scratch of lf_grad_noalloc: at most this many cells of a mesh in Morton
// order (8 Mi doubles, 64 MiB per GPU), on devices 0 .. kGradScratchDevices - 1
constexpr int64_t kGradScratchCells = int64_t(1) << 23;
constexpr int kGradScratchDevices = 64;


struct Rec {
    double x, y, z, w;
};

__device__ __forceinline__ Rec load_rec(const double *__restrict__ r, int64_t i) {
    const double2 *p = reinterpret_cast<const double2 *>(r + 4 * i);
    const double2 a = p[0], b = p[1];
    return Rec{a.x, a.y, b.x, b.y};
}

__device__ __forceinline__ void store_rec(double *__restrict__ r, int64_t i, double x, double y, double z,
                                          double w) {
    double2 *p = reinterpret_cast<double2 *>(r + 4 * i);
    p[0] = double2{x, y};
    p[1] = double2{z, w};
}

// Interpolation weights (Section 5.2, the weights loop): with the projected
// distances SfdOwn = |S_f.(C_f - C_P)| and SfdNei = |S_f.(C_N - C_f)|, the
// owner's weight is w_f = SfdNei / (SfdOwn + SfdNei), or 1/2 when
// |SfdOwn + SfdNei| does not exceed ROOTVSMALL (OpenFOAM's double-precision
// value, the square root of 1e-300).
//
// On a non-orthogonal mesh (gkface or gkband given) also the record of the
// Laplacian's correction: k_f = S_f/|S_f| - delta_f (C_N - C_P), with |S_f| and
// delta_f as the implicit part uses them, and the same weight.
constexpr double kRootVSmall = 1.0e-150;

__global__ void k_grad_face_geometry(int32_t f0, int32_t m, int32_t n, BandOffsets bo,
                                     const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
                                     const double *__restrict__ C, const double *__restrict__ S,
                                     const double *__restrict__ Cf, const double *__restrict__ mag_sf,
                                     const double *__restrict__ delta, double *__restrict__ gface,
                                     double *__restrict__ gband, double *__restrict__ gkface,
                                     double *__restrict__ gkband) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int64_t f = f0 + j;
    const double sx = S[3 * j], sy = S[3 * j + 1], sz = S[3 * j + 2];
    const double fx = Cf[3 * j], fy = Cf[3 * j + 1], fz = Cf[3 * j + 2];
    const double *P = C + 3 * static_cast<int64_t>(owner[f]);
    const double *Q = C + 3 * static_cast<int64_t>(neighbour[f]);
    const double sfd_own = fabs(sx * (fx - P[0]) + sy * (fy - P[1]) + sz * (fz - P[2]));
    const double sfd_nei = fabs(sx * (Q[0] - fx) + sy * (Q[1] - fy) + sz * (Q[2] - fz));
    const double den = sfd_own + sfd_nei;
    const double w = fabs(den) > kRootVSmall ? sfd_nei / den : 0.5;
    double kx = 0.0, ky = 0.0, kz = 0.0;
    if (gkface || gkband) {
        const double mg = mag_sf[f], dl = delta[f];
        kx = sx / mg - dl * (Q[0] - P[0]);
        ky = sy / mg - dl * (Q[1] - P[1]);
        kz = sz / mg - dl * (Q[2] - P[2]);
    }
    if (bo.k == 0) {
        store_rec(gface, f, sx, sy, sz, w);
        if (gkface) store_rec(gkface, f, kx, ky, kz, w);
        return;
    }
    const int32_t o = owner[f], off = neighbour[f] - o;
    for (int32_t k = 0; k < bo.k; ++k) {
        if (bo.d[k] == off) {
            store_rec(gband, static_cast<int64_t>(k) * n + o, sx, sy, sz, w);
            if (gkband) store_rec(gkband, static_cast<int64_t>(k) * n + o, kx, ky, kz, w);
        }
    }
}

__global__ void k_grad_bface_geometry(int32_t nb, const double *__restrict__ S, double *__restrict__ gbface) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double sx = S[3 * b], sy = S[3 * b + 1], sz = S[3 * b + 2];
    store_rec(gbface, b, sx, sy, sz, sqrt(sx * sx + sy * sy + sz * sz));
}

void launch_grad_face_geometry(int32_t f0, int32_t cnt, int32_t N, BandOffsets bo, const int32_t *owner,
                               const int32_t *neighbour, const double *C, const double *S, const double *Cf,
                               const double *mag_sf, const double *delta, double *gface, double *gband,
                               double *gkface, double *gkband, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_face_geometry, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, s, f0, cnt, N,
                       bo, owner, neighbour, C, S, Cf, mag_sf, delta, gface, gband, gkface, gkband);
}

void launch_grad_bface_geometry(int32_t nb, const double *bS, double *gbface, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_bface_geometry, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nb, bS,
                       gbface);
}

constexpr int kGradBlock = 256;

// Per-entry records of the row layout, one thread per solver row over exactly
// the entries of the row: the face's record, negated (area vector and weight)
// when the row's cell is the face's neighbour.  The weight is >= 0, so its sign
// bit tells the two kinds apart (-0.0 for a zero weight).
__global__ void k_grad_entry_geometry(int32_t n, const int32_t *__restrict__ soff, const int32_t *__restrict__ sface,
                                      const uint8_t *__restrict__ rlen, const int32_t *__restrict__ iperm,
                                      const int32_t *__restrict__ neighbour, const double *__restrict__ gface,
                                      double *__restrict__ gerec) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t mc = iperm ? iperm[r] : static_cast<int32_t>(r);
    int64_t idx = soff[r / kSlice] + r % kSlice;
    for (int32_t j = 0; j < rlen[r]; ++j, idx += kSlice) {
        const int32_t f = sface[idx];
        const Rec q = load_rec(gface, f);
        if (neighbour[f] == mc)
            store_rec(gerec, idx, -q.x, -q.y, -q.z, -q.w);
        else
            store_rec(gerec, idx, q.x, q.y, q.z, q.w);
    }
}

void launch_grad_entry_geometry(const lf_mesh *m, hipStream_t s) {
    const dim3 grid((m->N + kBlock - 1) / kBlock), block(kBlock);
    hipLaunchKernelGGL(k_grad_entry_geometry, grid, block, 0, s, m->N, m->soff, m->sface, m->rlen, m->iperm,
                       m->neighbour, m->gface, m->gerec);
    if (m->gkerec)
        hipLaunchKernelGGL(k_grad_entry_geometry, grid, block, 0, s, m->N, m->soff, m->sface, m->rlen, m->iperm,
                           m->neighbour, m->gkface, m->gkerec);
}

// the field in the solver's row order: Ts[r] = T[iperm[r]]
__global__ void k_grad_to_rows(int32_t n, const int32_t *__restrict__ iperm, const double *__restrict__ T,
                               double *__restrict__ Ts) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) Ts[r] = T[iperm[r]];
}

// the gradient back in the mesh's order: grad[c] = gs[perm[c]] (each thread
// gathers one row's three components and writes its cell's contiguously; a
// scatter of rows to their cells wrote partial cache lines at random)
__global__ void k_grad_from_rows(int32_t n, const int32_t *__restrict__ perm, const double *__restrict__ gs,
                                 double *__restrict__ grad) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t r = perm[c];
    const double gx = gs[3 * r], gy = gs[3 * r + 1], gz = gs[3 * r + 2];
    grad[3 * c] = gx;
    grad[3 * c + 1] = gy;
    grad[3 * c + 2] = gz;
}

// The internal faces' part of row r's gradient sum over its W slots of the
// row layout (W = the slice's width): every slot's record, column and
// neighbour value are loaded before any is used, so a thread has all its
// row's loads in flight at once; slots past the row's length (padding within
// the slice, in bounds) are loaded and skipped.  Terms are added in slot
// order, the order of the plain loop.
template <int W>
__device__ __forceinline__ void grad_row_faces(int64_t idx0, int32_t len, double Tr,
                                               const double *__restrict__ Ts, const int32_t *__restrict__ scol,
                                               const double *__restrict__ gerec, double &gx, double &gy,
                                               double &gz) {
    Rec q[W];
    int32_t col[W];
    double To[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        q[j] = load_rec(gerec, idx0 + static_cast<int64_t>(kSlice) * j);
        col[j] = scol[idx0 + static_cast<int64_t>(kSlice) * j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j) To[j] = Ts[col[j]];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j < len) {
            // lower face (negated record): s = w (T_P - T_r) + T_r, g -= S s;
            // owned face: s = w (T_r - T_N) + T_N, g += S s
            const double w = fabs(q[j].w);
            const double s = signbit(q[j].w) ? w * (To[j] - Tr) + Tr : w * (Tr - To[j]) + To[j];
            gx += q[j].x * s;
            gy += q[j].y * s;
            gz += q[j].z * s;
        }
    }
}

// Meshes without band form: one solver row per thread over the row layout,
// whose entries are the row's lower faces then its owned faces, each in
// ascending face order (the face loop's order); then the row's boundary faces
// ascending.  The field is read in the solver's order (Ts: T itself when the
// mesh keeps its order, else its copy in Morton order), so neighbours' values
// lie near the row; the gradient goes to the row's mesh cell.
__global__ void __launch_bounds__(kGradBlock)
k_grad_rows(int32_t n, const double *__restrict__ Ts, const double *__restrict__ Tb, const double *__restrict__ snb,
            const int32_t *__restrict__ soff, const int32_t *__restrict__ scol, const uint8_t *__restrict__ rlen,
            const double *__restrict__ gerec, const int32_t *__restrict__ rbface_start,
            const int32_t *__restrict__ rbface_list, const double *__restrict__ gbface,
            const double *__restrict__ V, const int32_t *__restrict__ iperm, double *__restrict__ grad,
            double *__restrict__ bgrad) {
    // iperm null: the gradient stays in the solver's order (or the orders agree)
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kGradBlock + threadIdx.x;
    if (r >= n) return;
    const int32_t o0 = soff[r / kSlice];
    const int64_t idx0 = o0 + r % kSlice;
    const int32_t width = (soff[r / kSlice + 1] - o0) / kSlice;
    const int32_t len = rlen[r];
    const double Tr = Ts[r];
    const double v = V[r];
    const int32_t b0 = rbface_start[r], b1 = rbface_start[r + 1];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    switch (width) {
        case 0: break;
        case 1: grad_row_faces<1>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        case 2: grad_row_faces<2>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        case 3: grad_row_faces<3>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        case 4: grad_row_faces<4>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        case 5: grad_row_faces<5>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        case 6: grad_row_faces<6>(idx0, len, Tr, Ts, scol, gerec, gx, gy, gz); break;
        default:
            for (int32_t j = 0; j < len; ++j) {
                const int64_t idx = idx0 + static_cast<int64_t>(kSlice) * j;
                const Rec q = load_rec(gerec, idx);
                const double To = Ts[scol[idx]];
                const double w = fabs(q.w);
                const double s = signbit(q.w) ? w * (To - Tr) + Tr : w * (Tr - To) + To;
                gx += q.x * s;
                gy += q.y * s;
                gz += q.z * s;
            }
    }
    for (int32_t k = b0; k < b1; ++k) {
        const int32_t b = rbface_list[k];
        const Rec q = load_rec(gbface, b);
        const double tb = Tb[b];
        gx += q.x * tb;
        gy += q.y * tb;
        gz += q.z * tb;
    }
    gx /= v;
    gy /= v;
    gz /= v;
    const int64_t c = iperm ? iperm[r] : r;
    grad[3 * c] = gx;
    grad[3 * c + 1] = gy;
    grad[3 * c + 2] = gz;
    if (!bgrad) return;
    // boundary value: g_b = g_c + n (snGrad_b - n.g_c), n = S_b / |S_b|
    for (int32_t k = b0; k < b1; ++k) {
        const int32_t b = rbface_list[k];
        const Rec q = load_rec(gbface, b);
        const double nx = q.x / q.w, ny = q.y / q.w, nz = q.z / q.w;
        const double d = snb[b] - (nx * gx + ny * gy + nz * gz);
        bgrad[3 * static_cast<int64_t>(b)] = gx + nx * d;
        bgrad[3 * static_cast<int64_t>(b) + 1] = gy + ny * d;
        bgrad[3 * static_cast<int64_t>(b) + 2] = gz + nz * d;
    }
}

// Workgroups are handed to the 8 dies (XCDs) in turn, each die with its own
// L2.  Renumbering them so that die x takes one contiguous run of cells keeps
// the face records a workgroup fetches in the L2 of the die that runs the
// next workgroups, which read them again one band offset later (at 256^3 this
// takes a fifth off the bytes fetched from beyond L2).
__device__ __forceinline__ int64_t die_block(unsigned b, unsigned nb) {
    const unsigned q = nb / kNumXcd, r = nb % kNumXcd, x = b % kNumXcd, i = b / kNumXcd;
    return static_cast<int64_t>(x) * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ bool is_face(const Rec &r) { return r.x != 0.0 || r.y != 0.0 || r.z != 0.0; }

// Band-form meshes: the faces of cell c are the band slots k*N + c (owned,
// neighbour c + d_k) and k*N + c - d_k (lower, owner c - d_k); a slot with a
// zero area vector holds no face (real faces have |S_f| > 0).  The lower
// faces are taken for k = K-1 .. 0 (ascending owner, i.e. ascending face
// index), the owned ones for k = 0 .. K-1 (ascending neighbour): the order of
// the face loop.  No lists are read for the internal faces, and every load
// is coalesced.
//
// Each thread walks R cells c, c + D, ..., c + (R-1) D along the widest band
// (D = d_{K-1}, one z layer of a box): the face it owns on that band is the
// next cell's lower face there, so its record and T[c] are carried in
// registers instead of being fetched again a whole layer later (by then out
// of L2 at 256^3).  Consecutive threads take consecutive c.  The caller's
// gradient (kStep false) goes to xyz rows grad[3c + i], written past the
// caches (a result for the caller, not read again here; 2% faster at 256^3);
// the corrected step's (kStep true) to one array per component, grad[i n + c],
// kept cached for the correction, which reads it next with contiguous loads.
template <int K, int R, bool kStep>
__global__ void __launch_bounds__(kGradBlock)
k_grad_band(int32_t n, BandOffsets bo, const double *__restrict__ T, const double *__restrict__ Tb,
            const double *__restrict__ snb, const double *__restrict__ gband,
            const int32_t *__restrict__ bface_start, const int32_t *__restrict__ bface_list,
            const double *__restrict__ gbface, const double *__restrict__ V, double *__restrict__ grad,
            double *__restrict__ bgrad) {
    const int64_t D = bo.d[K - 1];
    const int64_t g = die_block(blockIdx.x, gridDim.x) * kGradBlock + threadIdx.x;
    const int64_t chunk = g / D;
    int64_t c = chunk * R * D + (g - chunk * D);
    if (c >= n) return;
    const double *top = gband + 4 * static_cast<int64_t>(K - 1) * n;   // records of the widest band
    const Rec none{0.0, 0.0, 0.0, 0.0};
    Rec carry = c - D >= 0 ? load_rec(top, c - D) : none;   // lower face of c on the widest band
    double carry_T = c - D >= 0 ? T[c - D] : 0.0;
    double Tc = T[c];
#pragma unroll
    for (int r = 0; r < R; ++r, c += D) {
        if (c >= n) break;
        // everything the cell needs is requested up front, so one memory
        // latency covers the face records, T, V and the boundary-list range
        const double v = V[c];
        const int32_t b0 = bface_start[c], b1 = bface_start[c + 1];
        Rec lo[K], up[K];
        double Tlo[K], Tup[K];
        lo[K - 1] = carry;
        Tlo[K - 1] = carry_T;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t cl = c - bo.d[k], cu = c + bo.d[k];
            if (k < K - 1) {
                lo[k] = cl >= 0 ? load_rec(gband, static_cast<int64_t>(k) * n + cl) : none;
                Tlo[k] = cl >= 0 ? T[cl] : 0.0;
            }
            up[k] = cu < n ? load_rec(gband, static_cast<int64_t>(k) * n + c) : none;
            Tup[k] = cu < n ? T[cu] : 0.0;
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            if (is_face(lo[k])) {
                const double s = lo[k].w * (Tlo[k] - Tc) + Tc;
                gx -= lo[k].x * s;
                gy -= lo[k].y * s;
                gz -= lo[k].z * s;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (is_face(up[k])) {
                const double s = up[k].w * (Tc - Tup[k]) + Tup[k];
                gx += up[k].x * s;
                gy += up[k].y * s;
                gz += up[k].z * s;
            }
        }
        for (int32_t k = b0; k < b1; ++k) {
            const int32_t b = bface_list[k];
            const Rec rb = load_rec(gbface, b);
            const double tb = Tb[b];
            gx += rb.x * tb;
            gy += rb.y * tb;
            gz += rb.z * tb;
        }
        gx /= v;
        gy /= v;
        gz /= v;
        if (kStep) {
            grad[c] = gx;
            grad[n + c] = gy;
            grad[2 * static_cast<int64_t>(n) + c] = gz;
        } else {
            __builtin_nontemporal_store(gx, grad + 3 * c);
            __builtin_nontemporal_store(gy, grad + 3 * c + 1);
            __builtin_nontemporal_store(gz, grad + 3 * c + 2);
        }
        if (bgrad) {
            for (int32_t k = b0; k < b1; ++k) {
                const int32_t b = bface_list[k];
                const Rec rb = load_rec(gbface, b);
                const double nx = rb.x / rb.w, ny = rb.y / rb.w, nz = rb.z / rb.w;
                const double d = snb[b] - (nx * gx + ny * gy + nz * gz);
                bgrad[3 * static_cast<int64_t>(b)] = gx + nx * d;
                bgrad[3 * static_cast<int64_t>(b) + 1] = gy + ny * d;
                bgrad[3 * static_cast<int64_t>(b) + 2] = gz + nz * d;
            }
        }
        carry = up[K - 1];
        carry_T = Tc;
        Tc = Tup[K - 1];
    }
}

// Cells per thread of the band walk: 2 whenever the mesh has two layers.
// Longer walks fetch less (a quarter less at 256^3 with 8 cells than with 1)
// but keep fewer loads in flight, and at 256^3 they ran slower: 4 cells
// 2% and 8 cells 7% behind 2.
static int grad_walk_rows(int64_t n, int64_t D) { return n >= 2 * D ? 2 : 1; }

static int64_t grad_walk_groups(int64_t n, int64_t D, int R) {
    const int64_t threads = (n + R * D - 1) / (R * D) * D;
    return (threads + kGradBlock - 1) / kGradBlock;
}

static BandOffsets mesh_bands(const lf_mesh *m) {
    return BandOffsets{m->n_bands, {m->band_d[0], m->band_d[1], m->band_d[2], m->band_d[3]}};
}

// the band path's launch (1 <= n_bands <= 4, checked by the callers); step:
// the corrected step's gradient (one cached array per component), else the
// caller's (xyz rows written past the caches)
static void launch_grad_band(const lf_mesh *m, const double *T, const double *Tb, const double *snb, double *grad,
                             double *bgrad, bool step, hipStream_t s) {
    const BandOffsets bo = mesh_bands(m);
    const int K = bo.k;
    const int64_t D = bo.d[K - 1];
    const int R = grad_walk_rows(m->N, D);
    const dim3 grid(static_cast<unsigned>(grad_walk_groups(m->N, D, R))), block(kGradBlock);
#define LF_GRAD_BAND_NT(KK, RR, NT)                                                                      \
    if (K == KK && R == RR && step == NT)                                                                \
        hipLaunchKernelGGL((k_grad_band<KK, RR, NT>), grid, block, 0, s, m->N, bo, T, Tb, snb, m->gband,  \
                           m->bface_start, m->bface_list, m->gbface, m->V, grad, bgrad);
#define LF_GRAD_BAND(KK, RR) LF_GRAD_BAND_NT(KK, RR, false) LF_GRAD_BAND_NT(KK, RR, true)
#define LF_GRAD_BAND_R(KK) LF_GRAD_BAND(KK, 1) LF_GRAD_BAND(KK, 2)
    LF_GRAD_BAND_R(1)
    LF_GRAD_BAND_R(2)
    LF_GRAD_BAND_R(3)
    LF_GRAD_BAND_R(4)
#undef LF_GRAD_BAND_R
#undef LF_GRAD_BAND
#undef LF_GRAD_BAND_NT
}

// ---------------------------------------------------------------------------
// The Laplacian's explicit non-orthogonal correction (Gauss linear corrected
// scheme; the corrector loop around TEqn of Section 5.1 runs it once per step):
// face flux (DT |S_f|) (k_f . g_f) with g_f = w_f (g_P - g_N) + g_N, its
// divergence div_c = (owned faces' fluxes - lower faces' fluxes) / V_c summed
// in the face loop's order, and the laplacian's source 0 - V_c div_c, which the
// assembly subtracts from TEqn's source.  No boundary face contributes
// (k_b = 0 on non-coupled patches).
// ---------------------------------------------------------------------------

// T on the boundary faces: the fixed value, or the face cell's value
__global__ void k_nonorth_bvalues(int32_t nb, const int32_t *__restrict__ rbface_cell,
                                  const int32_t *__restrict__ bface_patch, const int32_t *__restrict__ patch_type,
                                  const double *__restrict__ patch_value, const double *__restrict__ T,
                                  double *__restrict__ Tb) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t pt = bface_patch[b];
    Tb[b] = patch_type[pt] == LF_BC_FIXED_VALUE ? patch_value[pt] : T[rbface_cell[b]];
}

// band-form meshes: a slot holds a face when its |S_f| > 0.  Launched like
// the gradient's band kernel: R cells per thread along the widest band, the
// shared face's record, |S_f| and the lower cell's gradient carried in
// registers, workgroups in die order.
template <int K, int R>
__global__ void __launch_bounds__(kGradBlock)
k_nonorth_band(int32_t n, BandOffsets bo, double DT, const double *__restrict__ g, const double *__restrict__ gkband,
               const double *__restrict__ band_mag_sf, const double *__restrict__ V, double *__restrict__ lap_src) {
    // g: one array per component (g[i n + c])
    const int64_t D = bo.d[K - 1];
    const int64_t t = die_block(blockIdx.x, gridDim.x) * kGradBlock + threadIdx.x;
    const int64_t chunk = t / D;
    int64_t c = chunk * R * D + (t - chunk * D);
    if (c >= n) return;
    const int64_t top = static_cast<int64_t>(K - 1) * n;     // slots of the widest band
    const Rec none{0.0, 0.0, 0.0, 0.0};
    Rec carry = none;
    double carry_mg = 0.0, carry_g[3] = {0.0, 0.0, 0.0};
    if (c - D >= 0) {
        carry = load_rec(gkband, top + c - D);
        carry_mg = band_mag_sf[top + c - D];
        for (int i = 0; i < 3; ++i) carry_g[i] = g[i * static_cast<int64_t>(n) + c - D];
    }
    double gc[3] = {g[c], g[n + c], g[2 * static_cast<int64_t>(n) + c]};
#pragma unroll
    for (int r = 0; r < R; ++r, c += D) {
        if (c >= n) break;
        const double v = V[c];
        Rec lo[K], up[K];
        double lmg[K], umg[K], glo[K][3], gup[K][3];
        lo[K - 1] = carry;
        lmg[K - 1] = carry_mg;
        for (int i = 0; i < 3; ++i) glo[K - 1][i] = carry_g[i];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t cl = c - bo.d[k], cu = c + bo.d[k];
            if (k < K - 1) {
                const bool in = cl >= 0;
                lo[k] = in ? load_rec(gkband, static_cast<int64_t>(k) * n + cl) : none;
                lmg[k] = in ? band_mag_sf[static_cast<int64_t>(k) * n + cl] : 0.0;
                for (int i = 0; i < 3; ++i) glo[k][i] = in ? g[i * static_cast<int64_t>(n) + cl] : 0.0;
            }
            const bool in = cu < n;
            up[k] = in ? load_rec(gkband, static_cast<int64_t>(k) * n + c) : none;
            umg[k] = in ? band_mag_sf[static_cast<int64_t>(k) * n + c] : 0.0;
            for (int i = 0; i < 3; ++i) gup[k][i] = in ? g[i * static_cast<int64_t>(n) + cu] : 0.0;
        }
        double div = 0.0;
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {      // lower faces (owner c - d_k): flux subtracted
            if (lmg[k] > 0.0) {
                const double fx = lo[k].w * (glo[k][0] - gc[0]) + gc[0];
                const double fy = lo[k].w * (glo[k][1] - gc[1]) + gc[1];
                const double fz = lo[k].w * (glo[k][2] - gc[2]) + gc[2];
                const double corr = lo[k].x * fx + lo[k].y * fy + lo[k].z * fz;
                div -= (DT * lmg[k]) * corr;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {           // owned faces (neighbour c + d_k): flux added
            if (umg[k] > 0.0) {
                const double fx = up[k].w * (gc[0] - gup[k][0]) + gup[k][0];
                const double fy = up[k].w * (gc[1] - gup[k][1]) + gup[k][1];
                const double fz = up[k].w * (gc[2] - gup[k][2]) + gup[k][2];
                const double corr = up[k].x * fx + up[k].y * fy + up[k].z * fz;
                div += (DT * umg[k]) * corr;
            }
        }
        div /= v;
        lap_src[c] = 0.0 - v * div;
        carry = up[K - 1];
        carry_mg = umg[K - 1];
        for (int i = 0; i < 3; ++i) {
            carry_g[i] = gc[i];
            gc[i] = gup[K - 1][i];
        }
    }
}

// one entry's correction flux: lower entries hold -k_f and -w_f, so their
// (negated) flux is added; the weight's sign bit picks the interpolation side
__device__ __forceinline__ double nonorth_entry(const Rec &q, double ox, double oy, double oz, double gx, double gy,
                                                double gz) {
    const double w = fabs(q.w);
    double fx, fy, fz;
    if (signbit(q.w)) {                     // lower face: g_f = w (g_o - g_r) + g_r
        fx = w * (ox - gx) + gx;
        fy = w * (oy - gy) + gy;
        fz = w * (oz - gz) + gz;
    } else {                                // owned face: g_f = w (g_r - g_o) + g_o
        fx = w * (gx - ox) + ox;
        fy = w * (gy - oy) + oy;
        fz = w * (gz - oz) + oz;
    }
    return q.x * fx + q.y * fy + q.z * fz;
}

// the row's W slots loaded before any is used (as grad_row_faces does), the
// fluxes added in slot order
template <int W>
__device__ __forceinline__ double nonorth_row_faces(int64_t idx0, int32_t len, double DT, double gx, double gy,
                                                    double gz, const double *__restrict__ g,
                                                    const int32_t *__restrict__ scol,
                                                    const double *__restrict__ gkerec,
                                                    const double *__restrict__ emag_sf) {
    Rec q[W];
    int32_t col[W];
    double mg[W], o[W][3];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int64_t idx = idx0 + static_cast<int64_t>(kSlice) * j;
        q[j] = load_rec(gkerec, idx);
        col[j] = scol[idx];
        mg[j] = emag_sf[idx];
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        for (int i = 0; i < 3; ++i) o[j][i] = g[3 * static_cast<int64_t>(col[j]) + i];
    double div = 0.0;
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (j < len) div += (DT * mg[j]) * nonorth_entry(q[j], o[j][0], o[j][1], o[j][2], gx, gy, gz);
    return div;
}

// row layout (solver order)
__global__ void __launch_bounds__(kGradBlock)
k_nonorth_rows(int32_t n, double DT, const double *__restrict__ g, const int32_t *__restrict__ soff,
               const int32_t *__restrict__ scol, const uint8_t *__restrict__ rlen, const double *__restrict__ gkerec,
               const double *__restrict__ emag_sf, const double *__restrict__ V, double *__restrict__ lap_src) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kGradBlock + threadIdx.x;
    if (r >= n) return;
    const int32_t o0 = soff[r / kSlice];
    const int64_t idx0 = o0 + r % kSlice;
    const int32_t width = (soff[r / kSlice + 1] - o0) / kSlice;
    const int32_t len = rlen[r];
    const double gx = g[3 * r], gy = g[3 * r + 1], gz = g[3 * r + 2];
    const double v = V[r];
    double div = 0.0;
    switch (width) {
        case 0: break;
        case 1: div = nonorth_row_faces<1>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        case 2: div = nonorth_row_faces<2>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        case 3: div = nonorth_row_faces<3>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        case 4: div = nonorth_row_faces<4>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        case 5: div = nonorth_row_faces<5>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        case 6: div = nonorth_row_faces<6>(idx0, len, DT, gx, gy, gz, g, scol, gkerec, emag_sf); break;
        default:
            for (int32_t j = 0; j < len; ++j) {
                const int64_t idx = idx0 + static_cast<int64_t>(kSlice) * j;
                const int64_t o = scol[idx];
                div += (DT * emag_sf[idx]) *
                       nonorth_entry(load_rec(gkerec, idx), g[3 * o], g[3 * o + 1], g[3 * o + 2], gx, gy, gz);
            }
    }
    div /= v;
    lap_src[r] = 0.0 - v * div;
}

void launch_nonorth_source(lf_problem *P, hipStream_t s, bool correction) {
    const lf_mesh *m = P->mesh;
    const dim3 block(kGradBlock), grid((m->N + kGradBlock - 1) / kGradBlock);
    if (m->B > 0)
        hipLaunchKernelGGL(k_nonorth_bvalues, dim3((m->B + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m->B,
                           m->rbface_cell, m->bface_patch, P->patch_type, P->patch_value, P->T, P->Tb);
    if (m->gkband) {
        {
            ProfScope ps(P, LF_K_GRAD, s);
            launch_grad_band(m, P->T, P->Tb, nullptr, P->grad3, nullptr, true, s);
        }
        if (!correction) return;
        const BandOffsets bo = mesh_bands(m);
        const int64_t D = bo.d[bo.k - 1];
        const int R = grad_walk_rows(m->N, D);
        const dim3 wgrid(static_cast<unsigned>(grad_walk_groups(m->N, D, R)));
#define LF_NONORTH_BAND(KK, RR)                                                                              \
        if (bo.k == KK && R == RR)                                                                           \
            LF_LAUNCH(P, LF_K_NONORTH, s, (k_nonorth_band<KK, RR>), wgrid, block, 0, s, m->N, bo, P->DT,     \
                      P->grad3, m->gkband, m->band_mag_sf, m->V, P->lap_src);
#define LF_NONORTH_BAND_R(KK) LF_NONORTH_BAND(KK, 1) LF_NONORTH_BAND(KK, 2)
        LF_NONORTH_BAND_R(1)
        LF_NONORTH_BAND_R(2)
        LF_NONORTH_BAND_R(3)
        LF_NONORTH_BAND_R(4)
#undef LF_NONORTH_BAND_R
#undef LF_NONORTH_BAND
    } else {
        // the gradient in the solver's order (T is kept in it): no copy, no scatter
        LF_LAUNCH(P, LF_K_GRAD, s, k_grad_rows, grid, block, 0, s, m->N, P->T, P->Tb, nullptr, m->soff, m->scol,
                  m->rlen, m->gerec, m->rbface_start, m->rbface_list, m->gbface, m->V, nullptr, P->grad3, nullptr);
        LF_LAUNCH(P, LF_K_NONORTH, s, k_nonorth_rows, grid, block, 0, s, m->N, P->DT, P->grad3, m->soff, m->scol,
                  m->rlen, m->gkerec, m->emag_sf, m->V, P->lap_src);
    }
}

// normal gradient of T on the boundary faces for the problem's conditions:
// fixedValue delta_b (T_b - T_P), zeroGradient 0
__global__ void k_bsngrad(int32_t nb, const int32_t *__restrict__ rbface_cell, const int32_t *__restrict__ bface_patch,
                          const int32_t *__restrict__ patch_type, const double *__restrict__ patch_value,
                          const double *__restrict__ bdelta, const double *__restrict__ T, double *__restrict__ snb) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t pt = bface_patch[b];
    snb[b] = patch_type[pt] == LF_BC_FIXED_VALUE ? bdelta[b] * (patch_value[pt] - T[rbface_cell[b]]) : 0.0;
}

// the gradient of the problem's T with its conditions (lf_problem_grad, whose
// argument and state checks come first)
lf_status launch_problem_grad(lf_problem *P, double *grad, double *bgrad) {
    const lf_mesh *m = P->mesh;
    if (!m->gface && !m->gband) {
        set_error("the mesh holds no gradient geometry (created without face centres)");
        return LF_EINVAL;
    }
    hipStream_t s = P->stream;
    if (m->B == 0) bgrad = nullptr;
    if (m->B > 0) {
        const dim3 bgrid((m->B + kBlock - 1) / kBlock), bblock(kBlock);
        hipLaunchKernelGGL(k_nonorth_bvalues, bgrid, bblock, 0, s, m->B, m->rbface_cell, m->bface_patch,
                           P->patch_type, P->patch_value, P->T, P->Tb);
        if (bgrad)
            hipLaunchKernelGGL(k_bsngrad, bgrid, bblock, 0, s, m->B, m->rbface_cell, m->bface_patch, P->patch_type,
                               P->patch_value, m->bdelta, P->T, P->snb);
    }
    if (m->gband) {
        if (m->n_bands < 1 || m->n_bands > kMaxBands) { set_error("bad band count %d", m->n_bands); return LF_EINVAL; }
        launch_grad_band(m, P->T, P->Tb, P->snb, grad, bgrad, false, s);
    } else {
        // T is kept in the solver's order: no copy; rows write to their mesh cells
        hipLaunchKernelGGL(k_grad_rows, dim3((m->N + kGradBlock - 1) / kGradBlock), dim3(kGradBlock), 0, s, m->N,
                           P->T, P->Tb, P->snb, m->soff, m->scol, m->rlen, m->gerec, m->rbface_start,
                           m->rbface_list, m->gbface, m->V, m->iperm, grad, bgrad);
    }
    LF_HIP(hipGetLastError());
    return LF_OK;
}

}  // namespace lf

using namespace lf;

extern "C" lf_status lf_grad(const lf_mesh *m, const double *T, const double *Tb, const double *snb, double *grad,
                             double *bgrad) {
    clear_error();
    if (!m || !T || !grad) { set_error("NULL argument"); return LF_EINVAL; }
    if (!m->gface && !m->gband) {
        set_error("the mesh holds no gradient geometry (created without face centres)");
        return LF_EINVAL;
    }
    if (m->B > 0 && !Tb) { set_error("Tb is NULL"); return LF_EINVAL; }
    if (m->B > 0 && bgrad && !snb) { set_error("snGrad_b is NULL while bgrad is given"); return LF_EINVAL; }
    if (m->B == 0) bgrad = nullptr;
    const dim3 block(kGradBlock);
    if (!m->gband) {
        const dim3 grid((m->N + kGradBlock - 1) / kGradBlock);
        if (!m->iperm) {
            hipLaunchKernelGGL(k_grad_rows, grid, block, 0, m->stream, m->N, T, Tb, snb, m->soff, m->scol, m->rlen,
                               m->gerec, m->rbface_start, m->rbface_list, m->gbface, m->V, nullptr, grad, bgrad);
        } else {
            // T into the solver's order, the gradient in it, then back to the mesh's order
            hipLaunchKernelGGL(k_grad_to_rows, grid, block, 0, m->stream, m->N, m->iperm, T, m->gT);
            hipLaunchKernelGGL(k_grad_rows, grid, block, 0, m->stream, m->N, m->gT, Tb, snb, m->soff, m->scol,
                               m->rlen, m->gerec, m->rbface_start, m->rbface_list, m->gbface, m->V, nullptr, m->gG,
                               bgrad);
            hipLaunchKernelGGL(k_grad_from_rows, grid, block, 0, m->stream, m->N, m->perm, m->gG, grad);
        }
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    if (m->n_bands < 1 || m->n_bands > kMaxBands) { set_error("bad band count %d", m->n_bands); return LF_EINVAL; }
    launch_grad_band(m, T, Tb, snb, grad, bgrad, false, m->stream);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

// ---------------------------------------------------------------------------
// lf_grad_noalloc: lf_grad for callers that cannot allocate device memory.
// Its one scratch buffer (T copied into the solver's order on a mesh kept in
// Morton order) is this file-scope array, one copy per GPU, held from the
// module's load until the process ends.  Host code reaches it only through
// the address hipGetSymbolAddress returns for that GPU (the array's name in
// host code is not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kGradScratchCells];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kGradScratchDevices] = {};

// the array's address on the current device (= dev), resolved once per device
lf_status grad_scratch(int dev, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kGradScratchDevices) {
        set_error("device %d is beyond the %d devices the scratch table covers", dev, kGradScratchDevices);
        return LF_EDEVICE;
    }
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return LF_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LF_OK;
}
}  // namespace

extern "C" lf_status lf_grad_noalloc(const lf_mesh *m, const double *T, const double *Tb, const double *snb,
                                     double *grad, double *bgrad) {
    clear_error();
    if (!m || !T || !grad) { set_error("NULL argument"); return LF_EINVAL; }
    if (!m->gface && !m->gband) {
        set_error("the mesh holds no gradient geometry (created without face centres)");
        return LF_EINVAL;
    }
    if (m->B > 0 && !Tb) { set_error("Tb is NULL"); return LF_EINVAL; }
    if (m->B > 0 && bgrad && !snb) { set_error("snGrad_b is NULL while bgrad is given"); return LF_EINVAL; }
    if (m->B == 0) bgrad = nullptr;
    if (m->gband) {
        // the band form reads T in place: no scratch
        if (m->n_bands < 1 || m->n_bands > kMaxBands) { set_error("bad band count %d", m->n_bands); return LF_EINVAL; }
        launch_grad_band(m, T, Tb, snb, grad, bgrad, false, m->stream);
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    const double *Ts = T;
    if (m->iperm) {
        if (static_cast<int64_t>(m->N) > kGradScratchCells) {
            set_error("lf_grad_noalloc: the mesh has %d cells in Morton order; its scratch holds at most %lld",
                      m->N, static_cast<long long>(kGradScratchCells));
            return LF_EINVAL;
        }
        int dev = -1;
        LF_HIP(hipGetDevice(&dev));
        if (dev != m->device) {
            set_error("lf_grad_noalloc: device %d is current, the mesh lives on %d", dev, m->device);
            return LF_EINVAL;
        }
        double *scr = nullptr;
        LF_TRY(grad_scratch(dev, &scr));
        const dim3 grid((m->N + kGradBlock - 1) / kGradBlock), block(kGradBlock);
        hipLaunchKernelGGL(k_grad_to_rows, grid, block, 0, m->stream, m->N, m->iperm, T, scr);
        Ts = scr;
    }
    hipLaunchKernelGGL(k_grad_rows, dim3((m->N + kGradBlock - 1) / kGradBlock), dim3(kGradBlock), 0, m->stream,
                       m->N, Ts, Tb, snb, m->soff, m->scol, m->rlen, m->gerec, m->rbface_start, m->rbface_list,
                       m->gbface, m->V, m->iperm, grad, bgrad);
    LF_HIP(hipGetLastError());
    return LF_OK;
}
