// Device helpers shared by the per-step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lf_problem.h"

namespace lf {

// Sum over a wavefront of 64 lanes by xor butterflies; every lane ends with the
// same value because each pairwise sum is commutative.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of NQ values over a workgroup of BS threads, result in every thread;
// fixed order (wave butterflies, then the wave sums in wave order).
template <int BS, int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ]) {
    constexpr int kWaves = BS / 64;
    __shared__ double red[NQ][kWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[q][wv] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = red[q][0];
#pragma unroll
        for (int j = 1; j < kWaves; ++j) s += red[q][j];
        v[q] = s;
    }
    __syncthreads();
}

// Rows of a launch with R rows per thread: workgroup b covers the R tiles of
// kCellBlock consecutive rows starting at row b * R * kCellBlock, thread t takes
// row t of each tile (each load of a wavefront stays one contiguous 64-row
// access, and a thread has R independent rows in flight).
template <int R>
__device__ __forceinline__ int32_t cell_row_at(int32_t blk, int j) {
    return (blk * R + j) * kCellBlock + static_cast<int32_t>(threadIdx.x);
}
template <int R>
__device__ __forceinline__ int32_t cell_row(int j) {
    return cell_row_at<R>(static_cast<int32_t>(blockIdx.x), j);
}

// first stage: the workgroup's partial sums go to part[slot * G + blockIdx.x]
// (BS: threads of the workgroup; _at: the workgroup's index blk within its
// problem's launch, for launches that serve several problems)
template <int NQ, int BS = kCellBlock>
__device__ __forceinline__ void write_partials_at(double *__restrict__ part, int32_t G, int32_t blk,
                                                  const int (&slot)[NQ], double (&v)[NQ]) {
    block_sum<BS, NQ>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[slot[q] * G + blk] = v[q];
    }
}
template <int NQ, int BS = kCellBlock>
__device__ __forceinline__ void write_partials(double *__restrict__ part, int32_t G, const int (&slot)[NQ],
                                               double (&v)[NQ]) {
    write_partials_at<NQ, BS>(part, G, static_cast<int32_t>(blockIdx.x), slot, v);
}

// second stage (one workgroup of kFinBlock threads): fixed-order sums of the
// first G partials of each slot (slots `stride` apart).  Thread t adds
// part[t], part[t + 1024], ... of each slot in that order; the loads of
// a group (kU per slot, every slot) are issued together, so the serial chain
// waits once per group: one or two groups at the sizes used here.
// (BS: the threads of the workgroup that sums; the result is in every thread)
template <int NQ, int BS = kFinBlock>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int32_t stride, int32_t G,
                                                const int (&slot)[NQ], double (&out)[NQ]) {
    constexpr int kU = NQ == 1 ? 32 : (NQ == 2 ? 16 : 8);
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] = 0.0;
    for (int32_t i0 = threadIdx.x; i0 < G; i0 += kU * BS) {
        double v[NQ][kU];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double *__restrict__ src = part + static_cast<int64_t>(slot[q]) * stride;
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                const int32_t i = i0 + j * BS;
                v[q][j] = i < G ? src[i] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int j = 0; j < kU; ++j) s[q] += v[q][j];
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = s[q];
    block_sum<BS, NQ>(out);
}

// the usual case: G partials per slot, slots G apart
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int32_t G, const int (&slot)[NQ],
                                                double (&out)[NQ]) {
    reduce_partials<NQ>(part, G, G, slot, out);
}

__device__ __forceinline__ bool check_conv(double res, double res0, double tol, double rel_tol) {
    return (res < tol) || (rel_tol > 1e-20 && res < rel_tol * res0);
}

// ---------------------------------------------------------------------------
// Rows of the sliced layout: entry j of row c at soff[c/64] + 64 j + c%64.
// Consecutive lanes hold consecutive rows, so each entry access of a
// wavefront is one contiguous 64-element load.  The slice width is the same
// for every lane of a wavefront, so the unrolled variants below load all of a
// row's entries first and then use them in order (padding entries are loaded
// but skipped: j >= len).
// ---------------------------------------------------------------------------
struct MeshRows {
    const int32_t *__restrict__ soff;
    const int32_t *__restrict__ scol;
    const int32_t *__restrict__ sface;
    const uint8_t *__restrict__ rlen;
};

// acc + sum_j a_j x[col_j] over the row's entries in order
template <int W, class T, class A>
__device__ __forceinline__ A row_dot_w(int32_t base, int32_t len, const int32_t *__restrict__ scol,
                                       const T *__restrict__ coef, const T *__restrict__ x, A acc) {
    int32_t col[W];
    T a[W], xv[W];
    // the row's column indices and coefficients are read once per product:
    // streamed past the caches, which then keep x for the gathers
#pragma unroll
    for (int j = 0; j < W; ++j) {
        col[j] = __builtin_nontemporal_load(&scol[base + kSlice * j]);
        a[j] = __builtin_nontemporal_load(&coef[base + kSlice * j]);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) xv[j] = x[col[j]];
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (j < len) acc += a[j] * xv[j];
    return acc;
}

template <class T, class A>
__device__ __forceinline__ A row_dot(const MeshRows &mr, int32_t c, const T *__restrict__ coef,
                                     const T *__restrict__ x, A acc) {
    const int32_t s = c >> 6;
    const int32_t o0 = mr.soff[s];
    const int32_t base = o0 + (c & (kSlice - 1));
    const int32_t width = (mr.soff[s + 1] - o0) >> 6;
    const int32_t len = mr.rlen[c];
    switch (width) {
        case 0: return acc;
        case 1: return row_dot_w<1>(base, len, mr.scol, coef, x, acc);
        case 2: return row_dot_w<2>(base, len, mr.scol, coef, x, acc);
        case 3: return row_dot_w<3>(base, len, mr.scol, coef, x, acc);
        case 4: return row_dot_w<4>(base, len, mr.scol, coef, x, acc);
        case 5: return row_dot_w<5>(base, len, mr.scol, coef, x, acc);
        case 6: return row_dot_w<6>(base, len, mr.scol, coef, x, acc);
        case 7: return row_dot_w<7>(base, len, mr.scol, coef, x, acc);
        case 8: return row_dot_w<8>(base, len, mr.scol, coef, x, acc);
        default: {
            int32_t idx = base;
            for (int32_t j = 0; j < len; ++j, idx += kSlice) acc += coef[idx] * x[mr.scol[idx]];
            return acc;
        }
    }
}

__device__ __forceinline__ int32_t row_base(const MeshRows &mr, int32_t c) {
    return mr.soff[c >> 6] + (c & (kSlice - 1));
}

// ---------------------------------------------------------------------------
// The two coefficient layouts of the per-step kernels.
//
// SellLayout: the sliced row layout above; each off-diagonal coefficient is
// stored in both of its rows, with its column index.
//
// BandLayout<K>: for meshes whose faces take only K offsets d_0 < ... <
// d_{K-1} (neighbour = owner + d_k), the coefficient of face (c, c + d_k) is
// stored once, at k*n + c (0 where that face does not exist).  Row c's
// entries are then the faces (c - d_k, c) for k = K-1 .. 0 (its lower faces,
// ascending column) followed by (c, c + d_k) for k = 0 .. K-1 (its owned
// faces, ascending column): the order of the sliced layout, so both layouts
// give the same sums (an absent face adds a zero term).  Columns are implicit
// and every access of a wavefront is contiguous.
// ---------------------------------------------------------------------------
struct SellLayout {
    MeshRows mr;
    const double *__restrict__ mag_sf;   // [F]
    const double *__restrict__ delta;    // [F]
    // the same factors per row entry, in the layout's order (null: gather by face)
    const double *__restrict__ emag_sf;  // [n_entries]
    const double *__restrict__ edelta;   // [n_entries]
};

template <int K>
struct BandLayout {
    int32_t n;
    int32_t d[K];
    const double *__restrict__ mag_sf;   // [K n], 0 where the face does not exist
    const double *__restrict__ delta;    // [K n]
};

// RBLayout: meshes with the two-colour band form (lf_mesh): the coefficient of
// the face of red cell u in direction d (-z, -y, -x, +x, +y, +z) is stored
// once, at d * nr + u.  A red row's entries are its six slots in that order
// (ascending black column); a black row's entries are the slots of its six
// red neighbours, mirrored (-z: red u - H, slot +z, ...), in ascending red
// column.  Both are the orders of the sliced layout, with absent faces as
// zero terms (a red row's own absent slot holds 0; a black row does not read
// a neighbour slot that belongs to another cell's face).
struct RBLayout {
    RBForm f;
    const double *__restrict__ mag_sf;   // [6 nr], 0 where the face does not exist
    const double *__restrict__ delta;    // [6 nr]
};

// One problem of a group launch (the work of several problems' steps in one
// launch per kernel): its parameters, layout (kind 0: the sliced rows mr with
// per-face and per-entry factors; K > 0: K bands with offsets d and per-slot
// factors), mesh arrays, boundary conditions and vectors.
struct MemberDesc {
    SolverParams sp;
    int32_t kind;
    int32_t n;
    int32_t d[4];
    int32_t diag_pc;
    double rdt, DT;
    MeshRows mr;
    const double *mag_sf, *delta, *emag_sf, *edelta;
    const int32_t *bface_start, *bface_list, *bface_patch;
    const double *bmag_sf, *bdelta, *V;
    const int32_t *patch_type;
    const double *patch_value;
    const int32_t *iperm;      // solver row -> mesh cell (null: the mesh's order)
    double *T, *coef, *diagB, *srcB, *r, *rD, *p;
    const float *coef32;
    float *coef32w, *sig32;
    float *r32, *p32, *d32, *q32;
    double *part;
    PcgState *st;
};

constexpr int kGroupMax = 32;   // problems of one group

// the members of one group launch: table slots and their first workgroups
// (begin[n] = the launch's workgroups)
struct GroupLaunch {
    int32_t n;
    int32_t slot[kGroupMax];
    int32_t begin[kGroupMax + 1];
};

// calls fn(layout) with a group member's layout object
template <class Fn>
__device__ __forceinline__ void with_member_layout(const MemberDesc &m, Fn &&fn) {
    switch (m.kind) {
        case 0: fn(SellLayout{m.mr, m.mag_sf, m.delta, m.emag_sf, m.edelta}); break;
        case 1: fn(BandLayout<1>{m.n, {m.d[0]}, m.mag_sf, m.delta}); break;
        case 2: fn(BandLayout<2>{m.n, {m.d[0], m.d[1]}, m.mag_sf, m.delta}); break;
        case 3: fn(BandLayout<3>{m.n, {m.d[0], m.d[1], m.d[2]}, m.mag_sf, m.delta}); break;
        default: fn(BandLayout<4>{m.n, {m.d[0], m.d[1], m.d[2], m.d[3]}, m.mag_sf, m.delta}); break;
    }
}

// the member of a group launch that workgroup b belongs to (members' first
// workgroups in gl.begin)
__device__ __forceinline__ int32_t group_member(const GroupLaunch &gl, int32_t b) {
    int32_t i = 0;
    while (i + 1 < gl.n && b >= gl.begin[i + 1]) ++i;
    return i;
}

// Row c's entries: coefficient slot, column and whether the entry may hold a
// face (else its term is zero; slot and column are then clamped in range)
__device__ __forceinline__ void rb_row(const RBForm &f, int32_t c, int64_t (&slot)[6], int32_t (&col)[6],
                                       bool (&ok)[6]) {
    const int32_t nr = f.nr;
    const bool red = c < nr;
    const int32_t u = red ? c : c - nr;
    const int32_t par = rb_par(f, u), pos = u % f.h;
    // the other colour's cell of each entry, in the row's order
    const int32_t o[6] = {u - f.H, u - f.h, red ? u + par - 1 : u - par, red ? u + par : u + 1 - par, u + f.h,
                          u + f.H};
    const bool xlo = red ? pos + par - 1 >= 0 : pos >= par;
    const bool xhi = red ? pos + par <= f.h - 1 : pos + 1 - par <= f.h - 1;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        bool v = o[j] >= 0 && o[j] < nr;
        if (j == 0 || j == 5) v = v && f.H > 0;
        if (j == 2) v = v && xlo;
        if (j == 3) v = v && xhi;
        ok[j] = v;
        const int32_t oc = v ? o[j] : u;
        // red: own slot of direction j; black: the red neighbour's mirrored slot
        slot[j] = static_cast<int64_t>(red ? j : 5 - j) * nr + (red ? u : oc);
        col[j] = red ? nr + oc : oc;
    }
}

// Both rows of half-index u (red cell u and black cell nr + u, neighbours in
// x on the box): entries as rb_row gives them, the line's parity computed once.
__device__ __forceinline__ void rb_pair(const RBForm &f, int32_t u, int64_t (&rslot)[6], int32_t (&rcol)[6],
                                        bool (&rok)[6], int64_t (&bslot)[6], int32_t (&bcol)[6],
                                        bool (&bok)[6]) {
    const int32_t nr = f.nr;
    const int32_t par = rb_par(f, u), pos = u % f.h;
    const int32_t ro[6] = {u - f.H, u - f.h, u + par - 1, u + par, u + f.h, u + f.H};
    const int32_t bo[6] = {u - f.H, u - f.h, u - par, u + 1 - par, u + f.h, u + f.H};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        bool vr = ro[j] >= 0 && ro[j] < nr, vb = bo[j] >= 0 && bo[j] < nr;
        if (j == 0 || j == 5) { vr = vr && f.H > 0; vb = vb && f.H > 0; }
        if (j == 2) { vr = vr && pos + par - 1 >= 0; vb = vb && pos >= par; }
        if (j == 3) { vr = vr && pos + par <= f.h - 1; vb = vb && pos + 1 - par <= f.h - 1; }
        rok[j] = vr;
        bok[j] = vb;
        rslot[j] = static_cast<int64_t>(j) * nr + u;
        rcol[j] = nr + (vr ? ro[j] : u);
        const int32_t ob = vb ? bo[j] : u;
        bslot[j] = static_cast<int64_t>(5 - j) * nr + ob;
        bcol[j] = ob;
    }
}

template <class T, class A>
__device__ __forceinline__ A layout_dot(const SellLayout &L, int32_t c, const T *__restrict__ coef,
                                        const T *__restrict__ x, A acc) {
    return row_dot(L.mr, c, coef, x, acc);
}

template <class T, class A>
__device__ __forceinline__ A layout_dot(const RBLayout &L, int32_t c, const T *__restrict__ coef,
                                        const T *__restrict__ x, A acc) {
    int64_t slot[6];
    int32_t col[6];
    bool ok[6];
    rb_row(L.f, c, slot, col, ok);
    T a[6], xv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const T v = coef[slot[j]];
        a[j] = ok[j] ? v : T(0);
        xv[j] = x[col[j]];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += a[j] * xv[j];
    return acc;
}

// acc + sum over the row's entries (order above) of a_j x[col_j]
template <int K, class T, class A>
__device__ __forceinline__ A layout_dot(const BandLayout<K> &L, int32_t c, const T *__restrict__ coef,
                                        const T *__restrict__ x, A acc) {
    T a[2 * K], xv[2 * K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int k = K - 1 - j;
        const bool ok = c >= L.d[k];
        const int32_t col = ok ? c - L.d[k] : c;
        const T v = coef[static_cast<int64_t>(k) * L.n + col];
        a[j] = ok ? v : T(0);
        xv[j] = x[col];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t col = c < L.n - L.d[k] ? c + L.d[k] : c;
        a[K + k] = coef[static_cast<int64_t>(k) * L.n + c];
        xv[K + k] = x[col];
    }
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) acc += a[j] * xv[j];
    return acc;
}

// ---------------------------------------------------------------------------
// Row walk over a band layout with K >= 2 bands.  The rows are cut into runs of
// kWalkRows * d1 consecutive rows (d1 = the second band's offset); thread t of
// run g takes the rows c0 = g kWalkRows d1 + t, c0 + d1, c0 + 2 d1, ...  A row's
// band-1 neighbours are then the thread's previous and next rows: their x
// values and the band-1 coefficient of the previous row stay in registers
// instead of being gathered again (on a box numbered x fastest these are the
// rows at -+nx, which for many rows lie in another workgroup, often on another
// XCD).  Each row's sum is layout_dot's, term for term in the same order, so
// the result is bitwise the same.
// ---------------------------------------------------------------------------
constexpr int kWalkRows = 8;
constexpr int kWalkMinBlocks = 2048;   // below this the flat one-row-per-thread launch is used

// workgroups of a walk launch over n rows with band-1 offset d1
inline int32_t walk_blocks(int32_t n, int32_t d1) {
    const int64_t run = static_cast<int64_t>(kWalkRows) * d1;
    const int64_t threads = (static_cast<int64_t>(n) + run - 1) / run * d1;
    return static_cast<int32_t>((threads + kCellBlock - 1) / kCellBlock);
}

// K when a layout can be walked (a band layout with K >= 2), else 0
template <class Lay>
struct WalkBands { static constexpr int value = 0; };
template <int K>
struct WalkBands<BandLayout<K>> { static constexpr int value = K >= 2 ? K : 0; };

// acc + the row's entries in layout_dot's order, with the band-1 lower entry
// (a_lo, x_lo) and the band-1 upper x value x_up supplied; a_up returns the
// row's own band-1 coefficient (the next row's lower one)
template <int K, class T, class A>
__device__ __forceinline__ A walk_row_dot(const BandLayout<K> &L, int64_t c, const T *__restrict__ coef,
                                          const T *__restrict__ x, A acc, T a_lo, T x_lo, T x_up, T &a_up) {
    static_assert(K >= 2, "the walk needs a second band");
    const int64_t n = L.n;
    T a[2 * K], xv[2 * K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int k = K - 1 - j;
        if (k == 1) {
            a[j] = a_lo;
            xv[j] = x_lo;
        } else {
            const bool ok = c >= L.d[k];
            const int64_t col = ok ? c - L.d[k] : c;
            const T v = coef[k * n + col];
            a[j] = ok ? v : T(0);
            xv[j] = x[col];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // the band-1 coefficient is read by this thread only (the next row
        // takes it from a register): stream it past the caches
        a[K + k] = k == 1 ? __builtin_nontemporal_load(&coef[k * n + c]) : coef[k * n + c];
        if (k == 1) {
            xv[K + k] = x_up;
        } else {
            const int64_t col = c < n - L.d[k] ? c + L.d[k] : c;
            xv[K + k] = x[col];
        }
    }
    a_up = a[K + 1];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) acc += a[j] * xv[j];
    return acc;
}

// The walk itself: calls fn(c, y_c, x_c, diag_c) for the thread's run rows in
// order, y = A x (diag x first, as layout_dot's callers do; kUnitDiag: a matrix
// with unit diagonal, x first, diag_c = 1).  kStream streams diag past the
// caches (it is touched once per launch).
template <int K, bool kStream, bool kUnitDiag, class T, class Fn>
__device__ __forceinline__ void band_walk_rows(const BandLayout<K> &L, const T *__restrict__ diag,
                                               const T *__restrict__ coef, const T *__restrict__ x, Fn &&fn) {
    const int64_t n = L.n, d1 = L.d[1];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x;
    const int64_t g = i / d1;
    int64_t c = g * kWalkRows * d1 + (i - g * d1);
    if (c >= n) return;
    T a_lo = T(0), x_lo;
    if (c >= d1) {
        a_lo = coef[n + c - d1];
        x_lo = x[c - d1];
    } else {
        x_lo = x[c];
    }
    T xc = x[c];
#pragma unroll
    for (int r = 0; r < kWalkRows; ++r) {
        if (c >= n) break;
        const T x_up = x[c < n - d1 ? c + d1 : c];
        T dc = T(1), acc = xc;
        if (!kUnitDiag) {
            dc = kStream ? __builtin_nontemporal_load(&diag[c]) : diag[c];
            acc = dc * xc;
        }
        T a_up;
        const T yc = walk_row_dot(L, c, coef, x, acc, a_lo, x_lo, x_up, a_up);
        fn(c, yc, xc, dc);
        a_lo = a_up;
        x_lo = xc;
        xc = x_up;
        c += d1;
    }
}

// y = A x by the walk; returns the FP64 sum over the thread's rows, in row
// order, of y_c x_c.  kStream also streams y past the caches.
template <int K, bool kStream, bool kUnitDiag, class T>
__device__ __forceinline__ double band_walk(const BandLayout<K> &L, const T *__restrict__ diag,
                                            const T *__restrict__ coef, const T *__restrict__ x,
                                            T *__restrict__ y) {
    double dot = 0.0;
    band_walk_rows<K, kStream, kUnitDiag>(L, diag, coef, x, [&](int64_t c, T yc, T xc, T) {
        if (kStream)
            __builtin_nontemporal_store(yc, &y[c]);
        else
            y[c] = yc;
        dot += static_cast<double>(yc) * static_cast<double>(xc);
    });
    return dot;
}


// ---------------------------------------------------------------------------
// Block walk over a box's band layout: three bands with offsets 1, nx, nx ny,
// i.e. row c = ix + nx iy + nx ny iz, with nx and N multiples of W.  The rows
// are cut into tiles of bw_lines(W) x-lines by bw_planes(W) planes; thread t
// of tile g takes
// the W x-adjacent rows c .. c + W - 1 (ix = W t) of each of the tile's
// lines, so every array is read 16 bytes per lane (W = 2 doubles, W = 4
// floats).  A row's y- and z-neighbours inside the thread's rows come from
// registers (the walk goes up the tile's lines: the upper line's values
// become the next row's own), its x-neighbours from the thread's other rows or
// from the adjacent lane when that lane holds the adjacent rows (same tile,
// which the lanes check once), else from memory.  Each row's sum is
// layout_dot's, term for term in the same order, so the product is bitwise
// the same; fewer, wider loads reach more of the HBM bandwidth than the
// one-row walk, whose neighbour gathers cost extra vector memory instructions.
// ---------------------------------------------------------------------------

// lane i takes v from lane i - 1 (lane 0: fill) / lane i + 1 (lane 63: fill)
// by the wavefront-wide DPP shifts; every lane of the wave must execute them
__device__ __forceinline__ int lane_from_below(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int lane_from_above(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float lane_from_below(float v) {
    return __int_as_float(lane_from_below(__float_as_int(v), 0));
}
__device__ __forceinline__ float lane_from_above(float v) {
    return __int_as_float(lane_from_above(__float_as_int(v), 0));
}
__device__ __forceinline__ double lane_from_below(double v) {
    return __hiloint2double(lane_from_below(__double2hiint(v), 0), lane_from_below(__double2loint(v), 0));
}
__device__ __forceinline__ double lane_from_above(double v) {
    return __hiloint2double(lane_from_above(__double2hiint(v), 0), lane_from_above(__double2loint(v), 0));
}

// W consecutive values, moved as one 16-byte access
template <class T, int W>
struct Lanes {
    static_assert(sizeof(T) * W == 16, "a lane moves 16 bytes");
    typedef T vec __attribute__((ext_vector_type(W)));
    T v[W];
};

template <class T, int W>
__device__ __forceinline__ Lanes<T, W> lanes_zero() {
    Lanes<T, W> r;
#pragma unroll
    for (int w = 0; w < W; ++w) r.v[w] = T(0);
    return r;
}

template <class T, int W, bool kStream = false>
__device__ __forceinline__ Lanes<T, W> lanes_load(const T *__restrict__ a, int64_t i) {
    typedef typename Lanes<T, W>::vec V;
    const V *p = reinterpret_cast<const V *>(a + i);
    const V x = kStream ? __builtin_nontemporal_load(p) : *p;
    Lanes<T, W> r;
#pragma unroll
    for (int w = 0; w < W; ++w) r.v[w] = x[w];
    return r;
}

template <class T, int W>
__device__ __forceinline__ void lanes_store_stream(T *__restrict__ a, int64_t i, const Lanes<T, W> &r) {
    typedef typename Lanes<T, W>::vec V;
    V x;
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = r.v[w];
    __builtin_nontemporal_store(x, reinterpret_cast<V *>(a + i));
}

// The product of the two-colour band layout with two red-black pairs per
// lane: lane t takes the pairs u = 2t and u + 1 (the same x-line, since h is
// even), so every array is read 16 bytes per lane (red slots, p of both
// colours, the diagonal; the y and z entries at u -+ h and u -+ H likewise).
// The x entries a pair's rows need from outside the lane's two pairs (p and
// the red slots +x and -x at u - 1 or u + 2) come from the adjacent lane when
// it holds the adjacent pairs, else from memory; a black row's x coefficients
// are its red neighbours' slots, which the lane has loaded as the red rows'
// own.  Each row's sum is the pair kernel's term for term (absent entries as
// zero coefficients times the row's own p), so the product is bitwise the
// same.  Every lane of a wave must run it (the lane exchanges).
inline bool rb2_form(const RBForm &f) { return f.h % 2 == 0 && f.nr % 2 == 0; }

inline int32_t rb2_blocks(int32_t nr) { return static_cast<int32_t>((nr / 2 + kCellBlock - 1) / kCellBlock); }

// a lane's pairs u, u + 1 and where their neighbours are: tv (the lane has
// pairs), the adjacent lanes holding pairs u - 2 and u + 2 (below_ok,
// above_ok), the line's parity and u's position in it, and which of the y and
// z neighbours exist (they are the same for both pairs, h and H being even)
struct Rb2Lane {
    int64_t u, pos;
    int32_t par;
    bool tv, below_ok, above_ok, zlo, zhi, ylo, yhi;
};

__device__ __forceinline__ Rb2Lane rb2_lane(const RBForm &f) {
    Rb2Lane l;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    l.u = 2 * (static_cast<int64_t>(blockIdx.x) * kCellBlock + threadIdx.x);
    l.tv = l.u < nr;
    const int key = l.tv ? static_cast<int>(l.u) : -8;
    l.below_ok = lane_from_below(key, -1000) == key - 2;
    l.above_ok = lane_from_above(key, -1000) == key + 2;
    l.par = l.tv ? rb_par(f, static_cast<int32_t>(l.u)) : 0;
    l.pos = l.tv ? l.u % h : 0;
    l.zlo = H > 0 && l.u >= H;
    l.zhi = H > 0 && l.u + H < nr;
    l.ylo = l.u >= h;
    l.yhi = l.u + h < nr;
    return l;
}

template <class Fn>
__device__ __forceinline__ void rb2_product(const RBForm &f, const double *__restrict__ diagB,
                                            const double *__restrict__ coef, const double *__restrict__ p,
                                            Fn &&fn) {
    typedef Lanes<double, 2> R;
    const int64_t nr = f.nr, h = f.h, H = f.H;
    const Rb2Lane l = rb2_lane(f);
    const int64_t u = l.u, pos = l.pos;
    const bool tv = l.tv, below_ok = l.below_ok, above_ok = l.above_ok;
    const int32_t par = l.par;
    const R z = lanes_zero<double, 2>();
    // own values: red slots 0..5, p of both colours, diagonals
    R sl[6], pr = z, pb = z, dr = z, db = z;
#pragma unroll
    for (int j = 0; j < 6; ++j) sl[j] = z;
    if (tv) {
#pragma unroll
        for (int j = 0; j < 6; ++j) sl[j] = lanes_load<double, 2>(coef, j * nr + u);
        pr = lanes_load<double, 2>(p, u);
        pb = lanes_load<double, 2>(p, nr + u);
        dr = lanes_load<double, 2, true>(diagB, u);
        db = lanes_load<double, 2, true>(diagB, nr + u);
    }
    // the adjacent lanes' values at u - 1 and u + 2 (p of both colours, the
    // red slots +x at u - 1 and -x at u + 2)
    double pb_m1 = lane_from_below(pb.v[1]), pr_m1 = lane_from_below(pr.v[1]), s3_m1 = lane_from_below(sl[3].v[1]);
    double pb_p2 = lane_from_above(pb.v[0]), pr_p2 = lane_from_above(pr.v[0]), s2_p2 = lane_from_above(sl[2].v[0]);
    if (!tv) return;
    if (!below_ok && pos >= 2) {
        pb_m1 = p[nr + u - 1];
        pr_m1 = p[u - 1];
        s3_m1 = coef[3 * nr + u - 1];
    }
    if (!above_ok && pos + 2 <= h - 1) {
        pb_p2 = p[nr + u + 2];
        pr_p2 = p[u + 2];
        s2_p2 = coef[2 * nr + u + 2];
    }
    // y and z entries: black p and the mirrored red slots (black rows) one
    // line or plane down and up, and the red p there
    const bool zlo = l.zlo, zhi = l.zhi, ylo = l.ylo, yhi = l.yhi;
    R pbz0 = z, pbz1 = z, pby0 = z, pby1 = z, prz0 = z, prz1 = z, pry0 = z, pry1 = z;
    R bz0 = z, bz1 = z, by0 = z, by1 = z;
    if (zlo) {
        pbz0 = lanes_load<double, 2>(p, nr + u - H);
        prz0 = lanes_load<double, 2>(p, u - H);
        bz0 = lanes_load<double, 2>(coef, 5 * nr + u - H);
    }
    if (ylo) {
        pby0 = lanes_load<double, 2>(p, nr + u - h);
        pry0 = lanes_load<double, 2>(p, u - h);
        by0 = lanes_load<double, 2>(coef, 4 * nr + u - h);
    }
    if (yhi) {
        pby1 = lanes_load<double, 2>(p, nr + u + h);
        pry1 = lanes_load<double, 2>(p, u + h);
        by1 = lanes_load<double, 2>(coef, nr + u + h);
    }
    if (zhi) {
        pbz1 = lanes_load<double, 2>(p, nr + u + H);
        prz1 = lanes_load<double, 2>(p, u + H);
        bz1 = lanes_load<double, 2>(coef, u + H);
    }
    R qr, qb;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int64_t pk = pos + k;
        // validity of the x entries (the pair kernel's rules)
        const bool rxlo = pk + par - 1 >= 0, rxhi = pk + par <= h - 1;
        const bool bxlo = pk >= par, bxhi = pk + 1 - par <= h - 1;
        // red row u + k: black p at u + k + par - 1 and u + k + par
        const double rpx_lo = par ? pb.v[k] : (k == 0 ? pb_m1 : pb.v[0]);
        const double rpx_hi = par ? (k == 0 ? pb.v[1] : pb_p2) : pb.v[k];
        // black row u + k: red p and the red slots -x / +x of the red cells at
        // u + k - par (its -x neighbour, slot +x) and u + k + 1 - par (slot -x)
        const double bpx_lo = par ? (k == 0 ? pr_m1 : pr.v[0]) : pr.v[k];
        const double bpx_hi = par ? pr.v[k] : (k == 0 ? pr.v[1] : pr_p2);
        const double bax_lo = par ? (k == 0 ? s3_m1 : sl[3].v[0]) : sl[3].v[k];
        const double bax_hi = par ? sl[2].v[k] : (k == 0 ? sl[2].v[1] : s2_p2);
        const double own_b = pb.v[k], own_r = pr.v[k];
        const double ra[6] = {zlo ? sl[0].v[k] : 0.0, ylo ? sl[1].v[k] : 0.0, rxlo ? sl[2].v[k] : 0.0,
                              rxhi ? sl[3].v[k] : 0.0, yhi ? sl[4].v[k] : 0.0, zhi ? sl[5].v[k] : 0.0};
        const double rx[6] = {zlo ? pbz0.v[k] : own_b, ylo ? pby0.v[k] : own_b, rxlo ? rpx_lo : own_b,
                              rxhi ? rpx_hi : own_b, yhi ? pby1.v[k] : own_b, zhi ? pbz1.v[k] : own_b};
        const double ba[6] = {zlo ? bz0.v[k] : 0.0, ylo ? by0.v[k] : 0.0, bxlo ? bax_lo : 0.0,
                              bxhi ? bax_hi : 0.0, yhi ? by1.v[k] : 0.0, zhi ? bz1.v[k] : 0.0};
        const double bx[6] = {zlo ? prz0.v[k] : own_r, ylo ? pry0.v[k] : own_r, bxlo ? bpx_lo : own_r,
                              bxhi ? bpx_hi : own_r, yhi ? pry1.v[k] : own_r, zhi ? prz1.v[k] : own_r};
        double a = dr.v[k] * pr.v[k], b = db.v[k] * pb.v[k];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            a += ra[j] * rx[j];
            b += ba[j] * bx[j];
        }
        qr.v[k] = a;
        qb.v[k] = b;
    }
    fn(u, qr, qb, pr, pb);
}

// The vector the walk multiplies: by default read from memory; a source may
// instead form each value from other arrays (vec(i): the W values at i, i a
// multiple of W; one(i): the value at i), as long as it gives the value the
// vector would hold.
template <class T, int W>
struct MemX {
    const T *__restrict__ x;
    __device__ __forceinline__ Lanes<T, W> vec(int64_t i) const { return lanes_load<T, W>(x, i); }
    __device__ __forceinline__ T one(int64_t i) const { return x[i]; }
};

// The walk: calls fn(c, y, x, diag) for the thread's groups of W rows
// (c .. c + W - 1; lines in order, within a line the planes in order), y = A x
// with the diagonal term first (kUnitDiag: a matrix with unit diagonal, x
// first, diag = 1, `diag` not read).  kStream streams diag past the caches.
// All lanes of a wave run the lane exchanges, so the caller must not branch
// around the call.
template <class T, int W, bool kStream, bool kUnitDiag, class XS, class Fn>
__device__ __forceinline__ void box_walk_xs(const BandLayout<3> &L, const BoxWalk &bw, const T *__restrict__ diag,
                                            const T *__restrict__ coef, const XS &x, Fn &&fn) {
    typedef Lanes<T, W> R;
    constexpr int kBwY = bw_lines(W), kBwZ = bw_planes(W);
    const int64_t n = L.n, d1 = L.d[1], d2 = L.d[2];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBwBlock + threadIdx.x;
    const int64_t g = i / bw.hx, t = i - g * bw.hx;
    const bool tv = g < bw.ntiles;
    const int64_t yb = g % bw.nyb, zb = g / bw.nyb;
    const int64_t iy0 = yb * kBwY;
    const int64_t base = W * t + d1 * iy0 + d2 * (zb * kBwZ);
    // the adjacent lanes hold the adjacent rows of every line iff their first
    // row is base -+ W (then they are threads t -+ 1 of the same tile)
    const int key = tv ? static_cast<int>(base) : -8;
    const bool below_ok = lane_from_below(key, -1000) == key - W;
    const bool above_ok = lane_from_above(key, -1000) == key + W;
    const R z = lanes_zero<T, W>();
    R xc[kBwZ], alo[kBwZ], xlo[kBwZ];
#pragma unroll
    for (int k = 0; k < kBwZ; ++k) {
        const int64_t c = base + k * d2;
        xc[k] = alo[k] = xlo[k] = z;
        if (tv && c < n) {
            xc[k] = x.vec(c);
            if (c >= d1) {
                alo[k] = lanes_load<T, W>(coef, n + c - d1);
                xlo[k] = x.vec(c - d1);
            } else {
                xlo[k] = xc[k];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kBwY; ++j) {
        const bool line = tv && iy0 + j < bw.ny;
        const int64_t c0 = base + j * d1;
        R xup[kBwZ], dg[kBwZ], a0[kBwZ], a1[kBwZ], a2[kBwZ];
        bool ok[kBwZ];
#pragma unroll
        for (int k = 0; k < kBwZ; ++k) {
            const int64_t c = c0 + k * d2;
            ok[k] = line && c < n;
            xup[k] = dg[k] = a0[k] = a1[k] = a2[k] = z;
            if (ok[k]) {
                xup[k] = x.vec(c < n - d1 ? c + d1 : c);
                if (!kUnitDiag) dg[k] = lanes_load<T, W, kStream>(diag, c);
                a0[k] = lanes_load<T, W>(coef, c);
                // the band-1 coefficient is read by this thread only (the next
                // line's row takes it from a register): stream it
                a1[k] = lanes_load<T, W, true>(coef, n + c);
                a2[k] = lanes_load<T, W>(coef, 2 * n + c);
            }
        }
        // z neighbours outside the tile: below its first plane, above its last
        R a2lo0 = z, xzlo0 = xc[0], xzhi_top = xc[kBwZ - 1];
        if (ok[0] && c0 >= d2) {
            a2lo0 = lanes_load<T, W>(coef, 2 * n + c0 - d2);
            xzlo0 = x.vec(c0 - d2);
        }
        {
            const int64_t ct = c0 + (kBwZ - 1) * d2;
            if (ok[kBwZ - 1] && ct < n - d2) xzhi_top = x.vec(ct + d2);
        }
#pragma unroll
        for (int k = 0; k < kBwZ; ++k) {
            const int64_t c = c0 + k * d2;
            // x neighbours across the lane's edges: row c's lower entry
            // (coefficient and x of c - 1) and row c + W - 1's upper x (c + W),
            // from the adjacent lanes when they hold them
            T a0lo = lane_from_below(a0[k].v[W - 1]), xm1 = lane_from_below(xc[k].v[W - 1]);
            T xpw = lane_from_above(xc[k].v[0]);
            if (ok[k] && !below_ok) {
                if (c >= 1) {
                    a0lo = coef[c - 1];
                    xm1 = x.one(c - 1);
                } else {
                    a0lo = T(0);
                    xm1 = xc[k].v[0];
                }
            }
            if (ok[k] && !above_ok) xpw = c < n - W ? x.one(c + W) : xc[k].v[W - 1];
            const R &a2lo = k == 0 ? a2lo0 : a2[k - 1];
            const R &xzlo = k == 0 ? xzlo0 : xc[k - 1];
            const R &xzhi = c < n - d2 ? (k + 1 < kBwZ ? xc[k + 1] : xzhi_top) : xc[k];
            R y;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                T acc = kUnitDiag ? xc[k].v[w] : dg[k].v[w] * xc[k].v[w];
                acc += a2lo.v[w] * xzlo.v[w];
                acc += alo[k].v[w] * xlo[k].v[w];
                acc += (w == 0 ? a0lo : a0[k].v[w - 1]) * (w == 0 ? xm1 : xc[k].v[w - 1]);
                acc += a0[k].v[w] * (w == W - 1 ? xpw : xc[k].v[w + 1]);
                acc += a1[k].v[w] * xup[k].v[w];
                acc += a2[k].v[w] * xzhi.v[w];
                y.v[w] = acc;
            }
            if (ok[k]) fn(c, y, xc[k], dg[k]);
        }
#pragma unroll
        for (int k = 0; k < kBwZ; ++k) {
            alo[k] = a1[k];
            xlo[k] = xc[k];
            xc[k] = xup[k];
        }
    }
}

template <class T, int W, bool kStream, bool kUnitDiag, class Fn>
__device__ __forceinline__ void box_walk(const BandLayout<3> &L, const BoxWalk &bw, const T *__restrict__ diag,
                                         const T *__restrict__ coef, const T *__restrict__ x, Fn &&fn) {
    box_walk_xs<T, W, kStream, kUnitDiag>(L, bw, diag, coef, MemX<T, W>{x}, fn);
}

// ---------------------------------------------------------------------------
// assembly (Listing 1): upper_f = -(delta_f (DT |S_f|)), diag = V/dt - lapDiag
// with lapDiag the negated sum of the Laplacian face coefficients of the row in
// face order, source = (T_old/dt) V; fixedValue faces add (DT|S_b|) delta_b to
// the diagonal and (DT|S_b|)(delta_b T_b) to the source.
// ---------------------------------------------------------------------------
// (edelta, emag_sf: the factors per entry, read contiguously; else gathered
// by face index)
template <int W, bool kUpper>
__device__ __forceinline__ double assemble_row_w(int32_t c, int32_t base, int32_t len, const MeshRows &mr,
                                                 const double *__restrict__ delta,
                                                 const double *__restrict__ mag_sf,
                                                 const double *__restrict__ edelta,
                                                 const double *__restrict__ emag_sf, double DT,
                                                 double *__restrict__ coef, double *__restrict__ upper) {
    int32_t f[W], col[W];
    double dl[W], ms[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        f[j] = mr.sface[base + kSlice * j];
        col[j] = mr.scol[base + kSlice * j];
    }
    if (edelta) {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            dl[j] = edelta[base + kSlice * j];
            ms[j] = emag_sf[base + kSlice * j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            dl[j] = delta[f[j]];
            ms[j] = mag_sf[f[j]];
        }
    }
    double lap_diag = 0.0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j < len) {
            const double lap_upper = dl[j] * (DT * ms[j]);
            coef[base + kSlice * j] = -lap_upper;
            lap_diag -= lap_upper;
            if (kUpper && col[j] > c) upper[f[j]] = -lap_upper;   // owned face: also in face order
        }
    }
    return lap_diag;
}

template <bool kUpper>
__device__ __forceinline__ double assemble_row(int32_t c, const MeshRows &mr, const double *__restrict__ delta,
                                               const double *__restrict__ mag_sf,
                                               const double *__restrict__ edelta,
                                               const double *__restrict__ emag_sf, double DT,
                                               double *__restrict__ coef, double *__restrict__ upper) {
    const int32_t s = c >> 6;
    const int32_t o0 = mr.soff[s];
    const int32_t base = o0 + (c & (kSlice - 1));
    const int32_t width = (mr.soff[s + 1] - o0) >> 6;
    const int32_t len = mr.rlen[c];
    switch (width) {
        case 0: return 0.0;
        case 1: return assemble_row_w<1, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 2: return assemble_row_w<2, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 3: return assemble_row_w<3, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 4: return assemble_row_w<4, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 5: return assemble_row_w<5, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 6: return assemble_row_w<6, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 7: return assemble_row_w<7, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        case 8: return assemble_row_w<8, kUpper>(c, base, len, mr, delta, mag_sf, edelta, emag_sf, DT, coef, upper);
        default: {
            double lap_diag = 0.0;
            int32_t idx = base;
            for (int32_t j = 0; j < len; ++j, idx += kSlice) {
                const int32_t f = mr.sface[idx];
                const double lap_upper = edelta ? edelta[idx] * (DT * emag_sf[idx]) : delta[f] * (DT * mag_sf[f]);
                coef[idx] = -lap_upper;
                lap_diag -= lap_upper;
                if (kUpper && mr.scol[idx] > c) upper[f] = -lap_upper;
            }
            return lap_diag;
        }
    }
}

// row product and row sum in one pass over the row's entries:
// ax = diag x_c + sum a_j x_j, sa = diag + sum a_j (both in entry order)
template <int W>
__device__ __forceinline__ void row_amul_sum_w(int32_t base, int32_t len, const int32_t *__restrict__ scol,
                                               const double *__restrict__ coef, const double *__restrict__ x,
                                               double &ax, double &sa) {
    int32_t col[W];
    double a[W], xv[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        col[j] = scol[base + kSlice * j];
        a[j] = coef[base + kSlice * j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j) xv[j] = x[col[j]];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j < len) {
            ax += a[j] * xv[j];
            sa += a[j];
        }
    }
}

__device__ __forceinline__ void row_amul_sum(const MeshRows &mr, int32_t c, const double *__restrict__ coef,
                                             const double *__restrict__ x, double &ax, double &sa) {
    const int32_t s = c >> 6;
    const int32_t o0 = mr.soff[s];
    const int32_t base = o0 + (c & (kSlice - 1));
    const int32_t width = (mr.soff[s + 1] - o0) >> 6;
    const int32_t len = mr.rlen[c];
    switch (width) {
        case 0: return;
        case 1: row_amul_sum_w<1>(base, len, mr.scol, coef, x, ax, sa); return;
        case 2: row_amul_sum_w<2>(base, len, mr.scol, coef, x, ax, sa); return;
        case 3: row_amul_sum_w<3>(base, len, mr.scol, coef, x, ax, sa); return;
        case 4: row_amul_sum_w<4>(base, len, mr.scol, coef, x, ax, sa); return;
        case 5: row_amul_sum_w<5>(base, len, mr.scol, coef, x, ax, sa); return;
        case 6: row_amul_sum_w<6>(base, len, mr.scol, coef, x, ax, sa); return;
        case 7: row_amul_sum_w<7>(base, len, mr.scol, coef, x, ax, sa); return;
        case 8: row_amul_sum_w<8>(base, len, mr.scol, coef, x, ax, sa); return;
        default: {
            int32_t idx = base;
            for (int32_t j = 0; j < len; ++j, idx += kSlice) {
                ax += coef[idx] * x[mr.scol[idx]];
                sa += coef[idx];
            }
        }
    }
}

// Layout-generic pieces of the assembly kernel.  RowCoefs keeps what the setup
// part needs of the row just assembled: the sliced layout re-reads the row it
// stored (only this thread writes it); the band layout keeps all 2K
// coefficients of the row in registers, since its lower coefficients live in
// other rows' slots, written by other threads of the same launch.
template <class Lay>
struct RowCoefs {};
template <int K>
struct RowCoefs<BandLayout<K>> {
    double a[2 * K];
};
template <>
struct RowCoefs<RBLayout> {
    double a[6];
    int32_t col[6];
};

template <bool kUpper>
__device__ __forceinline__ double assemble_coefs(const SellLayout &L, int32_t c, double DT,
                                                 double *__restrict__ coef, double *__restrict__ upper,
                                                 RowCoefs<SellLayout> &) {
    return assemble_row<kUpper>(c, L.mr, L.delta, L.mag_sf, L.edelta, L.emag_sf, DT, coef, upper);
}

// Band layout: the row's coefficients from the slot geometry (a slot without a
// face has zero factors, so its coefficient is zero and it leaves lapDiag
// unchanged); the row stores its owned faces' coefficients.  The face-order
// copy is written by a separate face kernel when asked for.
template <bool kUpper, int K>
__device__ __forceinline__ double assemble_coefs(const BandLayout<K> &L, int32_t c, double DT,
                                                 double *__restrict__ coef, double *__restrict__,
                                                 RowCoefs<BandLayout<K>> &rc) {
    double dl[2 * K], ms[2 * K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int k = K - 1 - j;
        const bool ok = c >= L.d[k];
        const int64_t slot = static_cast<int64_t>(k) * L.n + (ok ? c - L.d[k] : c);
        const double d0 = L.delta[slot], m0 = L.mag_sf[slot];
        dl[j] = ok ? d0 : 0.0;
        ms[j] = ok ? m0 : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t slot = static_cast<int64_t>(k) * L.n + c;
        dl[K + k] = L.delta[slot];
        ms[K + k] = L.mag_sf[slot];
    }
    double lap_diag = 0.0;
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) {
        const double lap_upper = dl[j] * (DT * ms[j]);
        rc.a[j] = -lap_upper;
        lap_diag -= lap_upper;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) coef[static_cast<int64_t>(k) * L.n + c] = rc.a[K + k];
    return lap_diag;
}

// Two-colour band form: a red row computes and stores its six slots; a black
// row computes its entries from the red neighbours' slot geometry (the same
// factors, so the same values) and stores nothing.
template <bool kUpper>
__device__ __forceinline__ double assemble_coefs(const RBLayout &L, int32_t c, double DT,
                                                 double *__restrict__ coef, double *__restrict__,
                                                 RowCoefs<RBLayout> &rc) {
    int64_t slot[6];
    bool ok[6];
    rb_row(L.f, c, slot, rc.col, ok);
    double dl[6], ms[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double d0 = L.delta[slot[j]], m0 = L.mag_sf[slot[j]];
        dl[j] = ok[j] ? d0 : 0.0;
        ms[j] = ok[j] ? m0 : 0.0;
    }
    double lap_diag = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double lap_upper = dl[j] * (DT * ms[j]);
        rc.a[j] = -lap_upper;
        lap_diag -= lap_upper;
    }
    if (c < L.f.nr) {
#pragma unroll
        for (int j = 0; j < 6; ++j) coef[slot[j]] = rc.a[j];
    }
    return lap_diag;
}

__device__ __forceinline__ void row_amul_sum(const RBLayout &, int32_t, const double *__restrict__,
                                             const RowCoefs<RBLayout> &rc, const double *__restrict__ x,
                                             double &ax, double &sa) {
    double xv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) xv[j] = x[rc.col[j]];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        ax += rc.a[j] * xv[j];
        sa += rc.a[j];
    }
}

__device__ __forceinline__ void store_coef32(const RBLayout &L, int32_t c, const double *__restrict__,
                                             const RowCoefs<RBLayout> &rc, float *__restrict__ coef32) {
    if (c >= L.f.nr) return;
#pragma unroll
    for (int j = 0; j < 6; ++j) coef32[static_cast<int64_t>(j) * L.f.nr + c] = static_cast<float>(rc.a[j]);
}

__device__ __forceinline__ void row_amul_sum(const SellLayout &L, int32_t c, const double *__restrict__ coef,
                                             const RowCoefs<SellLayout> &, const double *__restrict__ x,
                                             double &ax, double &sa) {
    row_amul_sum(L.mr, c, coef, x, ax, sa);
}

template <int K>
__device__ __forceinline__ void row_amul_sum(const BandLayout<K> &L, int32_t c, const double *__restrict__,
                                             const RowCoefs<BandLayout<K>> &rc, const double *__restrict__ x,
                                             double &ax, double &sa) {
    double xv[2 * K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int k = K - 1 - j;
        xv[j] = x[c >= L.d[k] ? c - L.d[k] : c];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) xv[K + k] = x[c < L.n - L.d[k] ? c + L.d[k] : c];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) {
        ax += rc.a[j] * xv[j];
        sa += rc.a[j];
    }
}

// FP32 copy of the row's stored coefficients (precision form)
__device__ __forceinline__ void store_coef32(const SellLayout &L, int32_t c, const double *__restrict__ coef,
                                             const RowCoefs<SellLayout> &, float *__restrict__ coef32) {
    int32_t idx = row_base(L.mr, c);
    const int32_t len = L.mr.rlen[c];
    for (int32_t j = 0; j < len; ++j, idx += kSlice) coef32[idx] = static_cast<float>(coef[idx]);
}

template <int K>
__device__ __forceinline__ void store_coef32(const BandLayout<K> &L, int32_t c, const double *__restrict__,
                                             const RowCoefs<BandLayout<K>> &rc, float *__restrict__ coef32) {
#pragma unroll
    for (int k = 0; k < K; ++k) coef32[static_cast<int64_t>(k) * L.n + c] = static_cast<float>(rc.a[K + k]);
}

}  // namespace lf
