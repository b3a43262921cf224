// Internal declarations of the lapfoam HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lapfoam.h"

namespace lf {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

// true while an lf_step_begin run of the problem has not finished
bool problem_in_flight(const lf_problem *P);

#define LF_HIP(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::lf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                            __FILE__, __LINE__);                                   \
            return LF_EDEVICE;                                                     \
        }                                                                          \
    } while (0)

#define LF_TRY(expr)                     \
    do {                                 \
        lf_status s_ = (expr);           \
        if (s_ != LF_OK) return s_;      \
    } while (0)

// ---------------------------------------------------------------------------
// workspace carving: a bump allocator over caller memory.  With base == nullptr
// it only counts, which is how the *_workspace_bytes functions size things.
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;

struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        used = (used + kAlign - 1) / kAlign * kAlign;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += sizeof(T) * (count ? count : 1);
        return p;
    }
    size_t bytes() const { return (used + kAlign - 1) / kAlign * kAlign; }
};

// ---------------------------------------------------------------------------
// launch geometry shared by the cell-parallel kernels
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;        // threads per workgroup of the mesh-build kernels
constexpr int kCellBlock = 512;    // threads per workgroup of the per-step kernels (one row each)
constexpr int kMxRows = 2;         // rows per thread of the precision form's FP32 inner kernels
constexpr int kUpdRows = 4;        // rows per thread of the FP64 update (diagonal preconditioner)
constexpr int kFinBlock = 1024;    // threads of the one-workgroup reduction kernels
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies
constexpr int kSlice = 64;         // rows per slice of the sliced row layout
constexpr int kMaxRowLen = 255;    // entries per row (stored as uint8)
constexpr int kMaxBands = 4;       // distinct neighbour - owner offsets of the band layout

// the band offsets of a mesh, passed to kernels by value
struct BandOffsets {
    int32_t k;
    int32_t d[kMaxBands];
};

// Two-colour band form of a mesh (see lf_mesh): nr cells of each colour, h per
// x-line, H per xy-plane (0: no third direction), ny lines per plane.
struct RBForm {
    int32_t nr, h, H, ny;
};

// parity of the line holding cell u of either colour
__host__ __device__ inline int32_t rb_par(const RBForm &f, int32_t u) {
    const int32_t line = u / f.h;
    return ((line % f.ny) + line / f.ny) & 1;
}

// direction 0..5 (-z, -y, -x, +x, +y, +z) of a face from red cell u to black
// cell nr + b, or -1 when no face of the form joins them
__host__ __device__ inline int32_t rb_direction(const RBForm &f, int32_t u, int32_t b) {
    const int32_t off = b - u;
    if (f.H > 0 && off == -f.H) return 0;
    if (off == -f.h) return 1;
    if (off == f.h) return 4;
    if (f.H > 0 && off == f.H) return 5;
    const int32_t par = rb_par(f, u), pos = u % f.h;
    if (off == par - 1 && pos + par - 1 >= 0) return 2;
    if (off == par && pos + par <= f.h - 1) return 3;
    return -1;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
}  // namespace lf

struct lf_mesh {
    int32_t N = 0, F = 0, P = 0, B = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool two_colour = false;    // max owner < min neighbour
    int32_t n_red = 0;          // first black cell when two_colour
    std::vector<int32_t> patch_start;   // host copy [P+1]
    // device arrays (inside the caller's workspace)
    int32_t *owner = nullptr, *neighbour = nullptr;       // [F]
    int32_t *owner_start = nullptr;                       // [N+1]
    int32_t *losort = nullptr, *losort_start = nullptr;   // [F], [N+1]
    int32_t *bface_start = nullptr, *bface_list = nullptr;   // [N+1], [B]
    int32_t *bface_cell = nullptr, *bface_patch = nullptr;   // [B]
    // Sliced row layout ("SELL-64"): rows grouped in slices of 64 consecutive
    // cells (one wavefront); slice s holds width_s entry columns stored
    // column-major, entry j of the row in lane l at soff[s] + 64 j + l.  A row's
    // entries are its lower faces (ascending) then its owned faces (ascending).
    int32_t n_slices = 0;
    int64_t n_entries = 0;
    int32_t *soff = nullptr;                              // [n_slices+1]
    int32_t *scol = nullptr, *sface = nullptr;            // [n_entries]
    uint8_t *rlen = nullptr;                              // [N] entries of each row
    // Band layout, when every internal face's offset neighbour - owner is one
    // of n_bands values band_d[0] < ... < band_d[n_bands-1] (a structured
    // numbering): the face (c, c + band_d[k]) has slot k*N + c, and the
    // geometry factors of each slot are stored there (0 where the face does
    // not exist).  n_bands = 0 when the mesh has no such form.
    int32_t n_bands = 0;
    int32_t band_d[lf::kMaxBands] = {0, 0, 0, 0};
    double *band_mag_sf = nullptr, *band_delta = nullptr; // [n_bands*N]
    // Two-colour band form: a box whose x-lines hold an even number of cells,
    // numbered red ((i+j+k) even) first, then black, each colour in natural
    // order.  A red cell u (and black cell n_red + u) then lies in line
    // u / rb_h of its colour, and its six neighbours of the other colour are
    // at u - rb_H, u - rb_h, u + par - 1, u + par, u + rb_h, u + rb_H with par
    // the line's parity ((line % rb_ny + line / rb_ny) & 1).  The face of red
    // cell u in direction d (0..5 in that order: -z, -y, -x, +x, +y, +z) has
    // slot d * n_red + u, whose geometry factors are stored there (0 where
    // the face does not exist).  rb_h = 0 when the mesh has no such form.
    int32_t rb_h = 0, rb_H = 0, rb_ny = 1;
    double *rb_mag_sf = nullptr, *rb_delta = nullptr;     // [6*n_red]
    // Box form: a band form with offsets 1, nx, nx*ny whose faces are those of
    // an nx x ny x nz box of hexahedra numbered i + nx (j + ny k) (none wraps
    // from one x-line or xy-plane into the next); 0 when not such a box.  The
    // multigrid preconditioner aggregates its 2 x 2 x 2 blocks.
    int32_t box_nx = 0, box_ny = 0, box_nz = 0;
    // Cell order of the solver's arrays.  Meshes without a band form and
    // without a two-colour numbering keep their cells in Morton order of the
    // cell centres (so that a row's neighbours lie near it in memory): the
    // solver's cell c is the mesh's cell iperm[c], and perm is the inverse.
    // Both are null when the mesh's own order is kept.  The lists of lists
    // above (owner_start, losort, bface_*) stay in the mesh's numbering; the
    // row layout, V and the rbface_* lists below are in the solver's order.
    int32_t *perm = nullptr, *iperm = nullptr;            // [N]
    int32_t *rbface_start = nullptr, *rbface_list = nullptr;   // [N+1], [B] boundary faces per solver row
    int32_t *rbface_cell = nullptr;                       // [B] solver row of each boundary face
    // |S_f| and delta_f per entry of the row layout (meshes without band form,
    // whose problems use that layout): the assembly reads them in row order
    double *emag_sf = nullptr, *edelta = nullptr;         // [n_entries], or null
    double *V = nullptr;                                  // [N] (solver order)
    double *mag_sf = nullptr, *delta = nullptr;           // [F]
    double *bmag_sf = nullptr, *bdelta = nullptr;         // [B]
    // Gauss gradient geometry (meshes created with face centres), in the
    // mesh's face order: per internal face {S_x, S_y, S_z, w_f} and per
    // boundary face {S_x, S_y, S_z, |S_b|}, 32 bytes each (two 16-byte loads)
    // On a mesh with band form the face records are kept by band slot
    // instead (gband, slot k*N + c for the face (c, c + band_d[k]), zero where
    // there is no such face) and gface is null.
    // Without band form the records are also kept per entry of the row layout
    // (gerec, in the solver's row order; an entry whose face has the row's cell
    // as neighbour stores -S_f and -w_f, the sign bit of w marking it), and
    // a reordered mesh keeps scratch copies of the field and its gradient in
    // the solver's order.
    double *gface = nullptr;                              // [4F], or null
    double *gerec = nullptr;                              // [4*n_entries], or null
    double *gT = nullptr;                                 // [N], or null
    double *gG = nullptr;                                 // [3N], or null
    double *gband = nullptr;                              // [4*n_bands*N], or null
    double *gbface = nullptr;                             // [4B], or null
    // Non-orthogonal meshes (LF_MESH_NON_ORTHOGONAL with face centres): the
    // Laplacian's correction records {k_x, k_y, k_z, w_f}, k_f = S_f/|S_f| -
    // delta_f (C_N - C_P), laid out like the gradient's (by band slot, or by
    // face and per row entry, negated for an entry whose row is the face's
    // neighbour)
    double *gkface = nullptr, *gkerec = nullptr, *gkband = nullptr;
    bool orthogonal = true;     // created without LF_MESH_NON_ORTHOGONAL
    size_t ws_bytes = 0;
};

struct lf_problem;   // defined in lf_problem.h

namespace lf {
// Gauss gradient geometry, built once per mesh (lf_grad.hip): the face records
// of faces [f0, f0 + cnt) from that chunk's area vectors S[3cnt] and centres
// Cf[3cnt] (cell centres C[3N]), stored at face f of gface, or, when bo.k > 0,
// at the face's band slot of gband (zeroed beforehand); the boundary-face
// records from S_b[3B]
void launch_grad_face_geometry(int32_t f0, int32_t cnt, int32_t N, BandOffsets bo, const int32_t *owner,
                               const int32_t *neighbour, const double *C, const double *S, const double *Cf,
                               const double *mag_sf, const double *delta, double *gface, double *gband,
                               double *gkface, double *gkband, hipStream_t s);
void launch_grad_bface_geometry(int32_t nb, const double *bS, double *gbface, hipStream_t s);
// the per-entry records gerec from the face records (after every chunk of them)
void launch_grad_entry_geometry(const lf_mesh *m, hipStream_t s);
}  // namespace lf
