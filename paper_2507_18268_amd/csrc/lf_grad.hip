// Gauss gradient of a cell field (Section 5.2: calcGrad = interpolate, gradf,
// correctBoundaryConditions), gathered per cell through the lists of lists.
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
#include "lf_internal.h"

namespace lf {

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
// owner's weight is w_f = SfdNei / (SfdOwn + SfdNei).
__global__ void k_grad_face_geometry(int32_t f0, int32_t m, const int32_t *__restrict__ owner,
                                     const int32_t *__restrict__ neighbour, const double *__restrict__ C,
                                     const double *__restrict__ S, const double *__restrict__ Cf,
                                     double *__restrict__ gface) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int64_t f = f0 + j;
    const double sx = S[3 * j], sy = S[3 * j + 1], sz = S[3 * j + 2];
    const double fx = Cf[3 * j], fy = Cf[3 * j + 1], fz = Cf[3 * j + 2];
    const double *P = C + 3 * static_cast<int64_t>(owner[f]);
    const double *Q = C + 3 * static_cast<int64_t>(neighbour[f]);
    const double sfd_own = fabs(sx * (fx - P[0]) + sy * (fy - P[1]) + sz * (fz - P[2]));
    const double sfd_nei = fabs(sx * (Q[0] - fx) + sy * (Q[1] - fy) + sz * (Q[2] - fz));
    store_rec(gface, f, sx, sy, sz, sfd_nei / (sfd_own + sfd_nei));
}

__global__ void k_grad_bface_geometry(int32_t nb, const double *__restrict__ S, double *__restrict__ gbface) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double sx = S[3 * b], sy = S[3 * b + 1], sz = S[3 * b + 2];
    store_rec(gbface, b, sx, sy, sz, sqrt(sx * sx + sy * sy + sz * sz));
}

void launch_grad_face_geometry(int32_t f0, int32_t cnt, const int32_t *owner, const int32_t *neighbour,
                               const double *C, const double *S, const double *Cf, double *gface,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_grad_face_geometry, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, s, f0, cnt,
                       owner, neighbour, C, S, Cf, gface);
}

void launch_grad_bface_geometry(int32_t nb, const double *bS, double *gbface, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_bface_geometry, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nb, bS,
                       gbface);
}

constexpr int kGradBlock = 256;

// One cell per thread, mesh order.  V is in the solver's order: V[vperm[c]]
// when the mesh keeps its cells reordered (vperm = perm), else V[c].
__global__ void __launch_bounds__(kGradBlock)
k_grad(int32_t n, const double *__restrict__ T, const double *__restrict__ Tb, const double *__restrict__ snb,
       const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
       const int32_t *__restrict__ owner_start, const int32_t *__restrict__ losort,
       const int32_t *__restrict__ losort_start, const int32_t *__restrict__ bface_start,
       const int32_t *__restrict__ bface_list, const double *__restrict__ gface,
       const double *__restrict__ gbface, const double *__restrict__ V, const int32_t *__restrict__ vperm,
       double *__restrict__ grad, double *__restrict__ bgrad) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kGradBlock + threadIdx.x;
    if (c >= n) return;
    const double Tc = T[c];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    // faces whose neighbour is c: s_f = w (T_P - T_c) + T_c, subtracted
    const int32_t l0 = losort_start[c], l1 = losort_start[c + 1];
    for (int32_t k = l0; k < l1; ++k) {
        const int32_t f = losort[k];
        const Rec r = load_rec(gface, f);
        const double s = r.w * (T[owner[f]] - Tc) + Tc;
        gx -= r.x * s;
        gy -= r.y * s;
        gz -= r.z * s;
    }
    // faces c owns: s_f = w (T_c - T_N) + T_N, added
    const int32_t o0 = owner_start[c], o1 = owner_start[c + 1];
    for (int32_t f = o0; f < o1; ++f) {
        const Rec r = load_rec(gface, f);
        const double TN = T[neighbour[f]];
        const double s = r.w * (Tc - TN) + TN;
        gx += r.x * s;
        gy += r.y * s;
        gz += r.z * s;
    }
    // boundary faces: S_b T_b, added
    const int32_t b0 = bface_start[c], b1 = bface_start[c + 1];
    for (int32_t k = b0; k < b1; ++k) {
        const int32_t b = bface_list[k];
        const Rec r = load_rec(gbface, b);
        const double tb = Tb[b];
        gx += r.x * tb;
        gy += r.y * tb;
        gz += r.z * tb;
    }
    const double v = V[vperm ? vperm[c] : c];
    gx /= v;
    gy /= v;
    gz /= v;
    grad[3 * c] = gx;
    grad[3 * c + 1] = gy;
    grad[3 * c + 2] = gz;
    if (!bgrad) return;
    // boundary value: g_b = g_c + n (snGrad_b - n.g_c), n = S_b / |S_b|
    for (int32_t k = b0; k < b1; ++k) {
        const int32_t b = bface_list[k];
        const Rec r = load_rec(gbface, b);
        const double nx = r.x / r.w, ny = r.y / r.w, nz = r.z / r.w;
        const double d = snb[b] - (nx * gx + ny * gy + nz * gz);
        bgrad[3 * static_cast<int64_t>(b)] = gx + nx * d;
        bgrad[3 * static_cast<int64_t>(b) + 1] = gy + ny * d;
        bgrad[3 * static_cast<int64_t>(b) + 2] = gz + nz * d;
    }
}

}  // namespace lf

using namespace lf;

extern "C" lf_status lf_grad(const lf_mesh *m, const double *T, const double *Tb, const double *snb, double *grad,
                             double *bgrad) {
    clear_error();
    if (!m || !T || !grad) { set_error("NULL argument"); return LF_EINVAL; }
    if (!m->gface) { set_error("the mesh holds no gradient geometry (created without face centres)"); return LF_EINVAL; }
    if (m->B > 0 && !Tb) { set_error("Tb is NULL"); return LF_EINVAL; }
    if (m->B > 0 && bgrad && !snb) { set_error("snGrad_b is NULL while bgrad is given"); return LF_EINVAL; }
    if (m->B == 0) bgrad = nullptr;
    hipLaunchKernelGGL(k_grad, dim3((m->N + kGradBlock - 1) / kGradBlock), dim3(kGradBlock), 0, m->stream, m->N, T,
                       Tb, snb, m->owner, m->neighbour, m->owner_start, m->losort, m->losort_start, m->bface_start,
                       m->bface_list, m->gface, m->gbface, m->V, m->perm, grad, bgrad);
    LF_HIP(hipGetLastError());
    return LF_OK;
}
