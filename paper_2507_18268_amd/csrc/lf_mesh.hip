// Mesh ingest: validation (host), the atomic-free "list of lists" addressing of
// Section 5.2 (GPU), the row-ordered off-diagonal layout used by every
// cell-parallel kernel (GPU) and the once-per-mesh geometry factors (GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "lf_internal.h"

namespace lf {

// ---------------------------------------------------------------------------
// errors (thread-local message)
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }

// ---------------------------------------------------------------------------
// integer kernels for the addressing build
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *a, int32_t n, int32_t v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// start[c] = first index i with key[i] >= c, for c in [0, n]; key sorted ascending.
__global__ void k_lower_bound_starts(const int32_t *__restrict__ key, int32_t m,
                                     int32_t *__restrict__ start, int32_t n) {
    int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c > n) return;
    int32_t lo = 0, hi = m;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (key[mid] < c) lo = mid + 1; else hi = mid;
    }
    start[c] = lo;
}

__global__ void k_histogram(const int32_t *__restrict__ key, int32_t m, int32_t *__restrict__ cnt) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) atomicAdd(&cnt[key[i]], 1);
}

// exclusive scan of cnt[n] into out[n+1] (out[n] = total), three passes
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t s[kBlock];
    int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int32_t add = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int32_t incl = s[t];
    *total = s[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_tile_sums(const int32_t *__restrict__ cnt, int32_t n,
                                                        int32_t *__restrict__ tile_sum) {
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int32_t v = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + threadIdx.x * kScanItems + j;
        if (i < n) v += cnt[i];
    }
    int32_t tot;
    block_exclusive_scan(v, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_tile_offsets(int32_t *tile_sum, int32_t nt) {
    int32_t carry = 0;
    for (int32_t base = 0; base < nt; base += kBlock) {
        int32_t i = base + threadIdx.x;
        int32_t v = i < nt ? tile_sum[i] : 0;
        int32_t tot;
        int32_t ex = block_exclusive_scan(v, &tot);
        if (i < nt) tile_sum[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int32_t *__restrict__ cnt, int32_t n,
                                                    const int32_t *__restrict__ tile_off,
                                                    int32_t *__restrict__ out) {
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int32_t loc[kScanItems];
    int32_t v = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        loc[j] = i < n ? cnt[i] : 0;
        v += loc[j];
    }
    int32_t tot;
    int32_t run = block_exclusive_scan(v, &tot) + tile_off[blockIdx.x];
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += loc[j];
        if (i == n - 1) out[n] = run;
    }
}

// place item i at start[key[i]] + slot (slot from an atomic counter), then
// sort each segment ascending so the result is the stable order.
__global__ void k_place(const int32_t *__restrict__ key, int32_t m, const int32_t *__restrict__ start,
                        int32_t *__restrict__ fill, int32_t *__restrict__ list) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t c = key[i];
    int32_t slot = atomicAdd(&fill[c], 1);
    list[start[c] + slot] = static_cast<int32_t>(i);
}

__global__ void k_sort_segments(const int32_t *__restrict__ start, int32_t n, int32_t *__restrict__ list) {
    int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    int32_t b = start[c], e = start[c + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t v = list[i];
        int32_t j = i - 1;
        while (j >= b && list[j] > v) {
            list[j + 1] = list[j];
            --j;
        }
        list[j + 1] = v;
    }
}

// Sliced row layout: row c lists its lower faces (ascending, the faces where c
// is the neighbour; column = owner) then its owned faces (ascending; column =
// neighbour).  On an upper-triangular mesh this is the order in which a
// sequential face loop visits row c.  Entry j of row c (slice s = c/64, lane
// l = c%64) sits at soff[s] + 64 j + l; entries past the row's length are
// padding (column = c, face = 0, coefficient 0): kernels may load them but
// never use them.
// With a cell order (perm/iperm, see lf_mesh), row r of the layout is the
// mesh's cell iperm[r], in the same face order, and columns are solver rows.
__global__ void k_sell_fill(int32_t n, const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
                            const int32_t *__restrict__ owner_start, const int32_t *__restrict__ losort,
                            const int32_t *__restrict__ losort_start, const int32_t *__restrict__ soff,
                            const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                            int32_t *__restrict__ scol, int32_t *__restrict__ sface, uint8_t *__restrict__ rlen) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t c = iperm ? iperm[r] : static_cast<int32_t>(r);
    const int32_t s = static_cast<int32_t>(r / kSlice), lane = static_cast<int32_t>(r % kSlice);
    const int32_t width = (soff[s + 1] - soff[s]) / kSlice;
    int32_t idx = soff[s] + lane, j = 0;
    // the host sized every slice from the same face counts; the j < width
    // guards only keep a disagreement from writing outside the slice
    for (int32_t i = losort_start[c]; i < losort_start[c + 1] && j < width; ++i, ++j, idx += kSlice) {
        const int32_t f = losort[i];
        scol[idx] = perm ? perm[owner[f]] : owner[f];
        sface[idx] = f;
    }
    for (int32_t f = owner_start[c]; f < owner_start[c + 1] && j < width; ++f, ++j, idx += kSlice) {
        scol[idx] = perm ? perm[neighbour[f]] : neighbour[f];
        sface[idx] = f;
    }
    rlen[r] = static_cast<uint8_t>(j);
    for (; j < width; ++j, idx += kSlice) {
        scol[idx] = static_cast<int32_t>(r);
        sface[idx] = 0;
    }
}

// Geometry factors (Gauss linear corrected Laplacian, orthogonal part):
// |S_f| and delta_f = 1/max(n.d, 0.05|d|), n = S_f/|S_f|, d = C_N - C_P.
__global__ void k_face_geometry(int32_t f0, int32_t m, const int32_t *__restrict__ owner,
                                const int32_t *__restrict__ neighbour, const double *__restrict__ C,
                                const double *__restrict__ S, double *__restrict__ mag_sf,
                                double *__restrict__ delta) {
    int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    int64_t f = f0 + j;
    double sx = S[3 * j], sy = S[3 * j + 1], sz = S[3 * j + 2];
    double mag = sqrt(sx * sx + sy * sy + sz * sz);
    double nx = sx / mag, ny = sy / mag, nz = sz / mag;
    const double *P = C + 3 * static_cast<int64_t>(owner[f]);
    const double *Q = C + 3 * static_cast<int64_t>(neighbour[f]);
    double dx = Q[0] - P[0], dy = Q[1] - P[1], dz = Q[2] - P[2];
    double nd = nx * dx + ny * dy + nz * dz;
    double dmag = sqrt(dx * dx + dy * dy + dz * dz);
    double lim = 0.05 * dmag;
    mag_sf[f] = mag;
    delta[f] = 1.0 / (nd > lim ? nd : lim);
}

// the face factors copied to each entry of the row layout, row by row over
// exactly the entries k_sell_fill wrote (padding entries copy face 0: loaded,
// never used; the lanes of a last, partial slice past the rows hold nothing)
__global__ void k_entry_geometry(int32_t n, const int32_t *__restrict__ soff, const int32_t *__restrict__ sface,
                                 const double *__restrict__ mag_sf, const double *__restrict__ delta,
                                 double *__restrict__ emag_sf, double *__restrict__ edelta) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t s = static_cast<int32_t>(r / kSlice), lane = static_cast<int32_t>(r % kSlice);
    const int32_t width = (soff[s + 1] - soff[s]) / kSlice;
    int32_t idx = soff[s] + lane;
    for (int32_t j = 0; j < width; ++j, idx += kSlice) {
        const int32_t f = sface[idx];
        emag_sf[idx] = mag_sf[f];
        edelta[idx] = delta[f];
    }
}

// boundary: |S_b| and delta_b = 1/(n_b.(C_b - C_P))
__global__ void k_bface_geometry(int32_t nb, const int32_t *__restrict__ bcell, const double *__restrict__ C,
                                 const double *__restrict__ S, const double *__restrict__ Cb,
                                 double *__restrict__ bmag, double *__restrict__ bdelta) {
    int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double sx = S[3 * b], sy = S[3 * b + 1], sz = S[3 * b + 2];
    double mag = sqrt(sx * sx + sy * sy + sz * sz);
    double nx = sx / mag, ny = sy / mag, nz = sz / mag;
    const double *P = C + 3 * static_cast<int64_t>(bcell[b]);
    double dx = Cb[3 * b] - P[0], dy = Cb[3 * b + 1] - P[1], dz = Cb[3 * b + 2] - P[2];
    double nd = nx * dx + ny * dy + nz * dz;
    bmag[b] = mag;
    bdelta[b] = 1.0 / nd;
}

// Band layout: the geometry factors of face f go to slot k*N + owner, k the
// index of its offset neighbour - owner among the mesh's band offsets (slots
// without a face keep the zeros written beforehand).
__global__ void k_fill_f64(double *a, int64_t n, double v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_band_fill(int32_t F, int32_t N, BandOffsets bo, const int32_t *__restrict__ owner,
                            const int32_t *__restrict__ neighbour, const double *__restrict__ mag_sf,
                            const double *__restrict__ delta, double *__restrict__ band_mag_sf,
                            double *__restrict__ band_delta) {
    int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t o = owner[f];
    const int32_t off = neighbour[f] - o;
    for (int32_t k = 0; k < bo.k; ++k) {
        if (bo.d[k] == off) {
            const int64_t slot = static_cast<int64_t>(k) * N + o;
            band_mag_sf[slot] = mag_sf[f];
            band_delta[slot] = delta[f];
        }
    }
}

// two-colour band form: the geometry factors of face (u, nr + b) at slot
// d * nr + u, d its direction (every face has one: checked on the host)
__global__ void k_rb_fill(int32_t F, RBForm rf, const int32_t *__restrict__ owner,
                          const int32_t *__restrict__ neighbour, const double *__restrict__ mag_sf,
                          const double *__restrict__ delta, double *__restrict__ rb_mag_sf,
                          double *__restrict__ rb_delta) {
    int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t u = owner[f];
    const int32_t d = rb_direction(rf, u, neighbour[f] - rf.nr);
    if (d < 0) return;
    const int64_t slot = static_cast<int64_t>(d) * rf.nr + u;
    rb_mag_sf[slot] = mag_sf[f];
    rb_delta[slot] = delta[f];
}

static inline unsigned blocks_for(int64_t n) {
    return static_cast<unsigned>((std::max<int64_t>(n, 1) + kBlock - 1) / kBlock);
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static constexpr int64_t kGeomChunk = 1 << 22;   // faces staged per geometry pass

struct MeshScratch {
    int32_t *cnt;        // [N+1]
    int32_t *tile;       // scan tile sums
    double *C;           // [3N]
    double *S;           // [3*chunk]
    double *bS, *bC;     // [3B]
    double *Cf;          // [3*chunk] face centres (gradient geometry only)
};

static void carve_mesh(Carver &cv, int32_t N, int32_t F, int32_t B, int64_t E, int32_t K, bool reorder,
                       bool grad, bool skew, int32_t rb_nr, lf_mesh *m, MeshScratch *s) {
    size_t n1 = static_cast<size_t>(N) + 1;
    const int32_t ns = (N + kSlice - 1) / kSlice;
    auto *owner = cv.take<int32_t>(F);
    auto *neighbour = cv.take<int32_t>(F);
    auto *owner_start = cv.take<int32_t>(n1);
    auto *losort = cv.take<int32_t>(F);
    auto *losort_start = cv.take<int32_t>(n1);
    auto *bface_start = cv.take<int32_t>(n1);
    auto *bface_list = cv.take<int32_t>(B);
    auto *bface_cell = cv.take<int32_t>(B);
    auto *bface_patch = cv.take<int32_t>(B);
    auto *soff = cv.take<int32_t>(static_cast<size_t>(ns) + 1);
    auto *scol = cv.take<int32_t>(static_cast<size_t>(E));
    auto *sface = cv.take<int32_t>(static_cast<size_t>(E));
    auto *rlen = cv.take<uint8_t>(N);
    auto *V = cv.take<double>(N);
    auto *mag_sf = cv.take<double>(F);
    auto *delta = cv.take<double>(F);
    auto *bmag = cv.take<double>(B);
    auto *bdelta = cv.take<double>(B);
    int32_t *perm = nullptr, *iperm = nullptr, *rbstart = bface_start, *rblist = bface_list, *rbcell = bface_cell;
    if (reorder) {
        perm = cv.take<int32_t>(N);
        iperm = cv.take<int32_t>(N);
        rbstart = cv.take<int32_t>(n1);
        rblist = cv.take<int32_t>(B);
        rbcell = cv.take<int32_t>(B);
    }
    double *emag = nullptr, *edelta = nullptr;
    if (K == 0 && E > 0) {
        emag = cv.take<double>(static_cast<size_t>(E));
        edelta = cv.take<double>(static_cast<size_t>(E));
    }
    double *band_mag = nullptr, *band_delta = nullptr;
    if (K > 0) {
        band_mag = cv.take<double>(static_cast<size_t>(K) * N);
        band_delta = cv.take<double>(static_cast<size_t>(K) * N);
    }
    double *rb_mag = nullptr, *rb_delta = nullptr;
    if (rb_nr > 0) {
        rb_mag = cv.take<double>(6 * static_cast<size_t>(rb_nr));
        rb_delta = cv.take<double>(6 * static_cast<size_t>(rb_nr));
    }
    double *gface = nullptr, *gband = nullptr, *gbface = nullptr, *gerec = nullptr, *gT = nullptr, *gG = nullptr;
    double *gkface = nullptr, *gkerec = nullptr, *gkband = nullptr;
    if (grad) {
        if (K > 0) {
            gband = cv.take<double>(4 * static_cast<size_t>(K) * N);
            if (skew) gkband = cv.take<double>(4 * static_cast<size_t>(K) * N);
        } else {
            gface = cv.take<double>(4 * static_cast<size_t>(F));
            gerec = cv.take<double>(4 * static_cast<size_t>(E));
            if (reorder) {
                gT = cv.take<double>(N);
                gG = cv.take<double>(3 * static_cast<size_t>(N));
            }
            if (skew) {
                gkface = cv.take<double>(4 * static_cast<size_t>(F));
                gkerec = cv.take<double>(4 * static_cast<size_t>(E));
            }
        }
        gbface = cv.take<double>(4 * static_cast<size_t>(B));
    }
    size_t tiles = (n1 + kScanTile - 1) / kScanTile + 1;
    MeshScratch sc;
    sc.cnt = cv.take<int32_t>(n1);
    sc.tile = cv.take<int32_t>(tiles);
    sc.C = cv.take<double>(3 * static_cast<size_t>(N));
    sc.S = cv.take<double>(3 * static_cast<size_t>(std::min<int64_t>(std::max(F, 1), kGeomChunk)));
    sc.bS = cv.take<double>(3 * static_cast<size_t>(B));
    sc.bC = cv.take<double>(3 * static_cast<size_t>(B));
    sc.Cf = grad ? cv.take<double>(3 * static_cast<size_t>(std::min<int64_t>(std::max(F, 1), kGeomChunk)))
                 : nullptr;
    if (m) {
        m->gface = gface; m->gband = gband; m->gbface = gbface; m->gerec = gerec; m->gT = gT; m->gG = gG;
        m->gkface = gkface; m->gkerec = gkerec; m->gkband = gkband;
        m->owner = owner; m->neighbour = neighbour; m->owner_start = owner_start;
        m->losort = losort; m->losort_start = losort_start; m->bface_start = bface_start;
        m->bface_list = bface_list; m->bface_cell = bface_cell; m->bface_patch = bface_patch;
        m->n_slices = ns; m->n_entries = E; m->soff = soff; m->scol = scol; m->sface = sface; m->rlen = rlen;
        m->V = V; m->mag_sf = mag_sf; m->delta = delta; m->bmag_sf = bmag; m->bdelta = bdelta;
        m->band_mag_sf = band_mag; m->band_delta = band_delta;
        m->rb_mag_sf = rb_mag; m->rb_delta = rb_delta;
        m->perm = perm; m->iperm = iperm;
        m->emag_sf = emag; m->edelta = edelta;
        m->rbface_start = rbstart; m->rbface_list = rblist; m->rbface_cell = rbcell;
    }
    if (s) *s = sc;
}

// Slice offsets of the row layout from the row lengths (faces per cell),
// counted on the host from the owner/neighbour lists: this only sizes the
// workspace; the entries themselves are filled on the GPU.
// With a cell order (iperm, solver row -> mesh cell) the rows are taken in
// that order; `bound` sizes every slice by the longest row instead (an upper
// bound for any order, used to size the workspace without the order).
static lf_status plan_slices(const lf_mesh_desc *d, const std::vector<int32_t> *iperm, bool bound,
                             std::vector<int32_t> *soff, int64_t *E) {
    const int32_t N = d->n_cells, F = d->n_faces;
    std::vector<int32_t> len(static_cast<size_t>(N), 0);
    for (int32_t f = 0; f < F; ++f) {
        const int32_t o = d->owner[f], n = d->neighbour[f];
        if (o >= 0 && o < N) ++len[o];
        if (n >= 0 && n < N) ++len[n];
    }
    int32_t longest = 0;
    for (int32_t c = 0; c < N; ++c) longest = std::max(longest, len[c]);
    const bool order = iperm && !iperm->empty();
    const int32_t ns = (N + kSlice - 1) / kSlice;
    if (soff) soff->assign(static_cast<size_t>(ns) + 1, 0);
    int64_t total = 0;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t w = bound ? longest : 0;
        if (!bound)
            for (int32_t r = s * kSlice; r < std::min(N, (s + 1) * kSlice); ++r)
                w = std::max(w, len[order ? (*iperm)[r] : r]);
        if (w > kMaxRowLen) {
            set_error("cell with %d faces: rows longer than %d are not supported", w, kMaxRowLen);
            return LF_EMESH;
        }
        total += static_cast<int64_t>(w) * kSlice;
        if (total > INT32_MAX) { set_error("mesh too large for 32-bit entry offsets"); return LF_EMESH; }
        if (soff) (*soff)[s + 1] = static_cast<int32_t>(total);
    }
    *E = total;
    return LF_OK;
}

// Band form: the distinct offsets neighbour - owner of the internal faces,
// ascending, when there are at most kMaxBands of them (a structured
// numbering, e.g. i + nx (j + ny k) on a block of hexahedra); else 0 bands.
static BandOffsets plan_bands(const lf_mesh_desc *d) {
    BandOffsets bo{};
    const int32_t F = d->n_faces;
    if (F <= 0 || !d->owner || !d->neighbour) return bo;
    int32_t k = 0;
    int32_t v[kMaxBands] = {0, 0, 0, 0};
    for (int32_t f = 0; f < F; ++f) {
        const int64_t off = static_cast<int64_t>(d->neighbour[f]) - d->owner[f];
        if (off <= 0 || off > INT32_MAX) return bo;
        bool seen = false;
        for (int32_t j = 0; j < k; ++j) seen = seen || v[j] == off;
        if (!seen) {
            if (k == kMaxBands) return bo;
            v[k++] = static_cast<int32_t>(off);
        }
    }
    std::sort(v, v + k);
    bo.k = k;
    for (int32_t j = 0; j < k; ++j) bo.d[j] = v[j];
    return bo;
}

// Box form (see lf_mesh): the band offsets 1, nx, nx*ny with N = nx ny nz
// (sides >= 2) and no face joining the end of an x-line or of an xy-plane to
// the start of the next one.
static void plan_box(const lf_mesh_desc *d, const BandOffsets &bo, int32_t dims[3]) {
    dims[0] = dims[1] = dims[2] = 0;
    const int32_t N = d->n_cells, F = d->n_faces;
    if (bo.k != 3 || bo.d[0] != 1 || bo.d[1] < 2 || bo.d[2] % bo.d[1] != 0 || N % bo.d[2] != 0) return;
    const int32_t nx = bo.d[1], ny = bo.d[2] / bo.d[1], nz = N / bo.d[2];
    if (ny < 2 || nz < 2) return;
    for (int32_t f = 0; f < F; ++f) {
        const int32_t c = d->owner[f], off = d->neighbour[f] - c;
        if (off == 1 && c % nx == nx - 1) return;
        if (off == nx && (c / nx) % ny == ny - 1) return;
    }
    dims[0] = nx; dims[1] = ny; dims[2] = nz;
}

// Two-colour band form (see lf_mesh): a two-colour numbering with as many red
// as black cells whose every face joins red cell u to black cell nr + b in
// one of the six directions of the form.  The per-line count h and per-plane
// count H are read off the offsets b - u of magnitude 2 or more (one
// magnitude: h, no third direction; none: a single line); every face is then
// checked against the form.  nr = 0 when the mesh does not have it.
static RBForm plan_rb(const lf_mesh_desc *d, bool two_colour, int32_t n_red) {
    RBForm none{0, 0, 0, 1};
    const int32_t N = d->n_cells, F = d->n_faces;
    if (!two_colour || F <= 0 || N % 2 != 0 || n_red != N / 2) return none;
    const int32_t nr = n_red;
    int64_t mags[2] = {0, 0};
    int nm = 0;
    for (int32_t f = 0; f < F; ++f) {
        const int64_t off = static_cast<int64_t>(d->neighbour[f]) - nr - d->owner[f];
        const int64_t a = off < 0 ? -off : off;
        if (a < 2) continue;
        if (nm > 0 && mags[0] == a) continue;
        if (nm > 1 && mags[1] == a) continue;
        if (nm == 2) return none;
        mags[nm++] = a;
    }
    if (nm == 2 && mags[0] > mags[1]) std::swap(mags[0], mags[1]);
    RBForm rf{nr, nm == 0 ? nr : static_cast<int32_t>(mags[0]), nm == 2 ? static_cast<int32_t>(mags[1]) : 0, 1};
    if (rf.h < 2 || nr % rf.h != 0) return none;
    if (rf.H > 0) {
        if (rf.H % rf.h != 0 || nr % rf.H != 0) return none;
        rf.ny = rf.H / rf.h;
    }
    for (int32_t f = 0; f < F; ++f)
        if (rb_direction(rf, d->owner[f], d->neighbour[f] - nr) < 0) return none;
    return rf;
}

// Cell order of the solver's arrays (see lf_mesh): for a mesh without band
// form and without a two-colour numbering, the cells sorted by the Morton
// (Z-order) key of their centres, 21 bits per axis over the bounding box,
// ties by cell index; empty (the mesh's own order) otherwise.
static uint64_t spread21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

static bool wants_cell_order(const lf_mesh_desc *d, int32_t n_bands, bool two_colour) {
    return n_bands == 0 && !two_colour && d->n_faces > 0 && d->n_cells > 1;
}

static std::vector<int32_t> plan_cell_order(const lf_mesh_desc *d) {
    const int32_t N = d->n_cells;
    const double *C = d->cell_centre;
    double lo[3] = {C[0], C[1], C[2]}, hi[3] = {C[0], C[1], C[2]};
    for (int32_t c = 1; c < N; ++c)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], C[3 * static_cast<int64_t>(c) + k]);
            hi[k] = std::max(hi[k], C[3 * static_cast<int64_t>(c) + k]);
        }
    std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(N));
    for (int32_t c = 0; c < N; ++c) {
        uint64_t z = 0;
        for (int k = 0; k < 3; ++k) {
            const double span = hi[k] - lo[k];
            double t = span > 0.0 ? (C[3 * static_cast<int64_t>(c) + k] - lo[k]) / span : 0.0;
            t = std::min(std::max(t, 0.0), 1.0);
            z |= spread21(static_cast<uint64_t>(t * 2097151.0)) << k;
        }
        key[c] = {z, c};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> iperm(static_cast<size_t>(N));
    for (int32_t r = 0; r < N; ++r) iperm[r] = key[r].second;
    return iperm;
}

// ---------------------------------------------------------------------------
// host validation
// ---------------------------------------------------------------------------
static lf_status validate(const lf_mesh_desc *d, int32_t *B_out, bool *two_colour, int32_t *n_red) {
    if (!d) { set_error("mesh desc is NULL"); return LF_EINVAL; }
    const int32_t N = d->n_cells, F = d->n_faces, P = d->n_patches;
    if (N < 1 || F < 0 || P < 0) { set_error("bad sizes N=%d F=%d P=%d", N, F, P); return LF_EINVAL; }
    if (!d->cell_volume || !d->cell_centre || (F > 0 && (!d->owner || !d->neighbour || !d->face_area)) ||
        !d->patch_start) {
        set_error("NULL mesh array");
        return LF_EINVAL;
    }
    if ((d->flags & ~LF_MESH_NON_ORTHOGONAL) != 0) { set_error("unknown mesh flags 0x%x", d->flags); return LF_EINVAL; }
    const bool skew_ok = (d->flags & LF_MESH_NON_ORTHOGONAL) != 0;
    if (d->patch_start[0] != 0) { set_error("patch_start[0] must be 0"); return LF_EMESH; }
    for (int32_t p = 0; p < P; ++p)
        if (d->patch_start[p + 1] < d->patch_start[p]) { set_error("patch_start not monotone"); return LF_EMESH; }
    const int32_t B = d->patch_start[P];
    if (B > 0 && (!d->bface_cell || !d->bface_area || !d->bface_centre)) {
        set_error("NULL boundary array");
        return LF_EINVAL;
    }
    for (int32_t c = 0; c < N; ++c)
        if (!(d->cell_volume[c] > 0.0) || !std::isfinite(d->cell_volume[c])) {
            set_error("cell %d: volume %g not positive/finite", c, d->cell_volume[c]);
            return LF_EMESH;
        }
    for (int64_t i = 0; i < 3 * static_cast<int64_t>(N); ++i)
        if (!std::isfinite(d->cell_centre[i])) { set_error("non-finite cell centre"); return LF_EMESH; }
    int32_t max_owner = -1, min_nei = N;
    for (int32_t f = 0; f < F; ++f) {
        int32_t o = d->owner[f], n = d->neighbour[f];
        if (o < 0 || o >= N || n < 0 || n >= N) { set_error("face %d: cell index out of range", f); return LF_EMESH; }
        if (o >= n) { set_error("face %d: owner %d >= neighbour %d", f, o, n); return LF_EMESH; }
        if (f > 0) {
            int32_t po = d->owner[f - 1], pn = d->neighbour[f - 1];
            if (o < po || (o == po && n <= pn)) {
                set_error("face %d: faces not in upper-triangular (owner, neighbour) order", f);
                return LF_EMESH;
            }
        }
        max_owner = std::max(max_owner, o);
        min_nei = std::min(min_nei, n);
        const double *S = d->face_area + 3 * static_cast<int64_t>(f);
        const double *A = d->cell_centre + 3 * static_cast<int64_t>(o);
        const double *Q = d->cell_centre + 3 * static_cast<int64_t>(n);
        double dx = Q[0] - A[0], dy = Q[1] - A[1], dz = Q[2] - A[2];
        double cx = S[1] * dz - S[2] * dy, cy = S[2] * dx - S[0] * dz, cz = S[0] * dy - S[1] * dx;
        double s2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
        double d2 = dx * dx + dy * dy + dz * dz;
        double sd = S[0] * dx + S[1] * dy + S[2] * dz;
        if (!(s2 > 0.0) || !(d2 > 0.0) || !std::isfinite(s2) || !(sd > 0.0) ||
            (!skew_ok && cx * cx + cy * cy + cz * cz > 1e-18 * s2 * d2)) {
            set_error("face %d: degenerate, inward or non-orthogonal face", f);
            return LF_EMESH;
        }
        if (d->face_centre) {
            const double *Cf = d->face_centre + 3 * static_cast<int64_t>(f);
            if (!std::isfinite(Cf[0]) || !std::isfinite(Cf[1]) || !std::isfinite(Cf[2])) {
                set_error("face %d: non-finite face centre", f);
                return LF_EMESH;
            }
        }
    }
    for (int32_t b = 0; b < B; ++b) {
        int32_t c = d->bface_cell[b];
        if (c < 0 || c >= N) { set_error("boundary face %d: cell out of range", b); return LF_EMESH; }
        const double *S = d->bface_area + 3 * static_cast<int64_t>(b);
        const double *Cb = d->bface_centre + 3 * static_cast<int64_t>(b);
        const double *A = d->cell_centre + 3 * static_cast<int64_t>(c);
        double sd = S[0] * (Cb[0] - A[0]) + S[1] * (Cb[1] - A[1]) + S[2] * (Cb[2] - A[2]);
        if (!(sd > 0.0) || !std::isfinite(sd)) {
            set_error("boundary face %d: not outward or degenerate", b);
            return LF_EMESH;
        }
    }
    *B_out = B;
    *two_colour = F > 0 && max_owner < min_nei;
    *n_red = F > 0 ? min_nei : N;
    return LF_OK;
}

static lf_status exclusive_scan(const int32_t *cnt, int32_t n, int32_t *out, int32_t *tile,
                                hipStream_t s) {
    int32_t nt = (n + kScanTile - 1) / kScanTile;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, out, 1, 0);
        LF_HIP(hipGetLastError());
        return LF_OK;
    }
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(nt), dim3(kBlock), 0, s, cnt, n, tile);
    hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(kBlock), 0, s, tile, nt);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kBlock), 0, s, cnt, n, tile, out);
    LF_HIP(hipGetLastError());
    return LF_OK;
}

// stable grouping of items 0..m-1 by key (key in [0, n)): start[n+1], list[m]
static lf_status group_by_key(const int32_t *key, int32_t m, int32_t n, int32_t *start, int32_t *list,
                              int32_t *cnt, int32_t *tile, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n + 1)), dim3(kBlock), 0, s, cnt, n + 1, 0);
    if (m > 0) hipLaunchKernelGGL(k_histogram, dim3(blocks_for(m)), dim3(kBlock), 0, s, key, m, cnt);
    LF_TRY(exclusive_scan(cnt, n, start, tile, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n + 1)), dim3(kBlock), 0, s, cnt, n + 1, 0);
    if (m > 0) {
        hipLaunchKernelGGL(k_place, dim3(blocks_for(m)), dim3(kBlock), 0, s, key, m, start, cnt, list);
        hipLaunchKernelGGL(k_sort_segments, dim3(blocks_for(n)), dim3(kBlock), 0, s, start, n, list);
    }
    LF_HIP(hipGetLastError());
    return LF_OK;
}

}  // namespace lf

using namespace lf;

extern "C" {

const char *lf_last_error(void) { return g_err; }

size_t lf_mesh_workspace_bytes(const lf_mesh_desc *d) {
    if (!d || d->n_cells < 1 || d->n_faces < 0 || d->n_patches < 0 || !d->patch_start) return 0;
    if (d->n_faces > 0 && (!d->owner || !d->neighbour)) return 0;
    const BandOffsets bo = plan_bands(d);
    // whether the cells are reordered depends on the two-colour test, which
    // needs the face lists only: the largest face owner against the smallest
    // neighbour
    int32_t max_owner = -1, min_nei = d->n_cells;
    for (int32_t f = 0; f < d->n_faces; ++f) {
        max_owner = std::max(max_owner, d->owner[f]);
        min_nei = std::min(min_nei, d->neighbour[f]);
    }
    const bool two_colour = d->n_faces > 0 && max_owner < min_nei;
    const bool reorder = wants_cell_order(d, bo.k, two_colour);
    const RBForm rf = plan_rb(d, two_colour, d->n_faces > 0 ? min_nei : d->n_cells);
    int64_t E = 0;
    if (plan_slices(d, nullptr, reorder, nullptr, &E) != LF_OK) return 0;
    Carver cv(nullptr);
    carve_mesh(cv, d->n_cells, d->n_faces, d->patch_start[d->n_patches], E, bo.k, reorder,
               d->face_centre != nullptr, (d->flags & LF_MESH_NON_ORTHOGONAL) != 0, rf.nr, nullptr, nullptr);
    return cv.bytes();
}

lf_status lf_mesh_create(const lf_mesh_desc *d, void *ws, size_t ws_bytes, void *stream, lf_mesh **out) {
    clear_error();
    if (!out) { set_error("out is NULL"); return LF_EINVAL; }
    *out = nullptr;
    int32_t B = 0, n_red = 0;
    bool two_colour = false;
    LF_TRY(validate(d, &B, &two_colour, &n_red));
    const int32_t N = d->n_cells, F = d->n_faces, P = d->n_patches;
    const BandOffsets bo = plan_bands(d);
    const bool reorder = wants_cell_order(d, bo.k, two_colour);
    const RBForm rf = plan_rb(d, two_colour, n_red);
    std::vector<int32_t> iperm_h;
    if (reorder) iperm_h = plan_cell_order(d);
    std::vector<int32_t> soff_h;
    int64_t E = 0;
    LF_TRY(plan_slices(d, &iperm_h, false, &soff_h, &E));
    const bool grad = d->face_centre != nullptr;
    const bool skew = (d->flags & LF_MESH_NON_ORTHOGONAL) != 0;
    Carver dry(nullptr);
    carve_mesh(dry, N, F, B, E, bo.k, reorder, grad, skew, rf.nr, nullptr, nullptr);
    if (!ws || ws_bytes < dry.bytes() || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
        set_error("mesh workspace too small or misaligned: need %zu bytes, 256-aligned", dry.bytes());
        return LF_ENOMEM;
    }
    lf_mesh *m = new (std::nothrow) lf_mesh();
    if (!m) { set_error("host allocation failed"); return LF_ENOMEM; }
    m->N = N; m->F = F; m->P = P; m->B = B;
    m->two_colour = two_colour;
    m->n_red = n_red;
    m->n_bands = bo.k;
    for (int32_t k = 0; k < bo.k; ++k) m->band_d[k] = bo.d[k];
    m->stream = static_cast<hipStream_t>(stream);
    m->patch_start.assign(d->patch_start, d->patch_start + P + 1);
    m->ws_bytes = dry.bytes();
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; set_error("hipGetDevice failed"); return LF_EDEVICE; }
    Carver cv(ws);
    MeshScratch sc;
    carve_mesh(cv, N, F, B, E, bo.k, reorder, grad, skew, rf.nr, m, &sc);
    if (rf.nr > 0) { m->rb_h = rf.h; m->rb_H = rf.H; m->rb_ny = rf.ny; }
    {
        int32_t dims[3];
        plan_box(d, bo, dims);
        m->box_nx = dims[0]; m->box_ny = dims[1]; m->box_nz = dims[2];
    }
    m->orthogonal = (d->flags & LF_MESH_NON_ORTHOGONAL) == 0;
    hipStream_t s = m->stream;

    auto fail = [&](lf_status st) { delete m; return st; };
    std::vector<int32_t> bpatch(static_cast<size_t>(B));
    for (int32_t p = 0; p < P; ++p)
        for (int32_t b = d->patch_start[p]; b < d->patch_start[p + 1]; ++b) bpatch[b] = p;

#define LF_HIPM(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                   \
            return fail(LF_EDEVICE);                                                    \
        }                                                                               \
    } while (0)

    if (F > 0) {
        LF_HIPM(hipMemcpyAsync(m->owner, d->owner, sizeof(int32_t) * F, hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(m->neighbour, d->neighbour, sizeof(int32_t) * F, hipMemcpyHostToDevice, s));
    }
    LF_HIPM(hipMemcpyAsync(m->soff, soff_h.data(), sizeof(int32_t) * soff_h.size(), hipMemcpyHostToDevice, s));
    std::vector<int32_t> perm_h, rbcell_h;
    std::vector<double> V_h;
    if (reorder) {
        perm_h.resize(static_cast<size_t>(N));
        for (int32_t r = 0; r < N; ++r) perm_h[iperm_h[r]] = r;
        V_h.resize(static_cast<size_t>(N));
        for (int32_t r = 0; r < N; ++r) V_h[r] = d->cell_volume[iperm_h[r]];
        rbcell_h.resize(static_cast<size_t>(B));
        for (int32_t b = 0; b < B; ++b) rbcell_h[b] = perm_h[d->bface_cell[b]];
        LF_HIPM(hipMemcpyAsync(m->perm, perm_h.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(m->iperm, iperm_h.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(m->V, V_h.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        if (B > 0)
            LF_HIPM(hipMemcpyAsync(m->rbface_cell, rbcell_h.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    } else {
        LF_HIPM(hipMemcpyAsync(m->V, d->cell_volume, sizeof(double) * N, hipMemcpyHostToDevice, s));
    }
    LF_HIPM(hipMemcpyAsync(sc.C, d->cell_centre, sizeof(double) * 3 * static_cast<size_t>(N),
                           hipMemcpyHostToDevice, s));
    if (B > 0) {
        LF_HIPM(hipMemcpyAsync(m->bface_cell, d->bface_cell, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(m->bface_patch, bpatch.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(sc.bS, d->bface_area, sizeof(double) * 3 * static_cast<size_t>(B),
                               hipMemcpyHostToDevice, s));
        LF_HIPM(hipMemcpyAsync(sc.bC, d->bface_centre, sizeof(double) * 3 * static_cast<size_t>(B),
                               hipMemcpyHostToDevice, s));
    }

    // lists of lists (Section 5.2): owned faces, lower faces, boundary faces per cell
    hipLaunchKernelGGL(k_lower_bound_starts, dim3(blocks_for(static_cast<int64_t>(N) + 1)), dim3(kBlock), 0, s,
                       m->owner, F, m->owner_start, N);
    lf_status st = group_by_key(m->neighbour, F, N, m->losort_start, m->losort, sc.cnt, sc.tile, s);
    if (st != LF_OK) return fail(st);
    st = group_by_key(m->bface_cell, B, N, m->bface_start, m->bface_list, sc.cnt, sc.tile, s);
    if (st != LF_OK) return fail(st);
    if (reorder) {
        // the same boundary lists, per solver row
        st = group_by_key(m->rbface_cell, B, N, m->rbface_start, m->rbface_list, sc.cnt, sc.tile, s);
        if (st != LF_OK) return fail(st);
    }
    hipLaunchKernelGGL(k_sell_fill, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, m->owner, m->neighbour,
                       m->owner_start, m->losort, m->losort_start, m->soff, m->perm, m->iperm, m->scol, m->sface,
                       m->rlen);

    // geometry factors, faces staged in chunks
    if (m->gband) {
        const int64_t slots = 4 * static_cast<int64_t>(bo.k) * N;
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->gband, slots, 0.0);
        if (m->gkband)
            hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->gkband, slots, 0.0);
    }
    for (int64_t f0 = 0; f0 < F; f0 += kGeomChunk) {
        int32_t cnt = static_cast<int32_t>(std::min<int64_t>(kGeomChunk, F - f0));
        LF_HIPM(hipMemcpyAsync(sc.S, d->face_area + 3 * f0, sizeof(double) * 3 * static_cast<size_t>(cnt),
                               hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_face_geometry, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, static_cast<int32_t>(f0),
                           cnt, m->owner, m->neighbour, sc.C, sc.S, m->mag_sf, m->delta);
        if (grad) {
            LF_HIPM(hipMemcpyAsync(sc.Cf, d->face_centre + 3 * f0, sizeof(double) * 3 * static_cast<size_t>(cnt),
                                   hipMemcpyHostToDevice, s));
            launch_grad_face_geometry(static_cast<int32_t>(f0), cnt, N, bo, m->owner, m->neighbour, sc.C, sc.S,
                                      sc.Cf, m->mag_sf, m->delta, m->gface, m->gband, m->gkface, m->gkband, s);
        }
    }
    if (bo.k > 0) {
        const int64_t slots = static_cast<int64_t>(bo.k) * N;
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->band_mag_sf, slots, 0.0);
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->band_delta, slots, 0.0);
        hipLaunchKernelGGL(k_band_fill, dim3(blocks_for(F)), dim3(kBlock), 0, s, F, N, bo, m->owner, m->neighbour,
                           m->mag_sf, m->delta, m->band_mag_sf, m->band_delta);
    }
    if (rf.nr > 0) {
        const int64_t slots = 6 * static_cast<int64_t>(rf.nr);
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->rb_mag_sf, slots, 0.0);
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(slots)), dim3(kBlock), 0, s, m->rb_delta, slots, 0.0);
        hipLaunchKernelGGL(k_rb_fill, dim3(blocks_for(F)), dim3(kBlock), 0, s, F, rf, m->owner, m->neighbour,
                           m->mag_sf, m->delta, m->rb_mag_sf, m->rb_delta);
    }
    if (m->emag_sf)
        hipLaunchKernelGGL(k_entry_geometry, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, m->soff, m->sface,
                           m->mag_sf, m->delta, m->emag_sf, m->edelta);
    if (B > 0)
        hipLaunchKernelGGL(k_bface_geometry, dim3(blocks_for(B)), dim3(kBlock), 0, s, B, m->bface_cell, sc.C,
                           sc.bS, sc.bC, m->bmag_sf, m->bdelta);
    if (grad && B > 0) launch_grad_bface_geometry(B, sc.bS, m->gbface, s);
    if (m->gerec) launch_grad_entry_geometry(m, s);
    LF_HIPM(hipGetLastError());
    LF_HIPM(hipStreamSynchronize(s));
#undef LF_HIPM
    *out = m;
    return LF_OK;
}

lf_status lf_mesh_bands(const lf_mesh *m, int32_t *n_bands, int32_t *offsets) {
    clear_error();
    if (!m || !n_bands) { set_error("NULL argument"); return LF_EINVAL; }
    *n_bands = m->n_bands;
    if (offsets)
        for (int32_t k = 0; k < kMaxBands; ++k) offsets[k] = k < m->n_bands ? m->band_d[k] : 0;
    return LF_OK;
}

lf_status lf_mesh_cell_order(const lf_mesh *m, int32_t *reordered, int32_t *order) {
    clear_error();
    if (!m || !reordered) { set_error("NULL argument"); return LF_EINVAL; }
    *reordered = m->iperm ? 1 : 0;
    if (order) {
        if (m->iperm) {
            LF_HIP(hipMemcpyAsync(order, m->iperm, sizeof(int32_t) * m->N, hipMemcpyDeviceToHost, m->stream));
            LF_HIP(hipStreamSynchronize(m->stream));
        } else {
            for (int32_t c = 0; c < m->N; ++c) order[c] = c;
        }
    }
    return LF_OK;
}

lf_status lf_mesh_destroy(lf_mesh *m) {
    delete m;
    return LF_OK;
}

lf_status lf_mesh_get_addressing(const lf_mesh *m, int32_t *owner_start, int32_t *losort, int32_t *losort_start,
                                 int32_t *bface_start, int32_t *bface_list) {
    clear_error();
    if (!m) { set_error("mesh is NULL"); return LF_EINVAL; }
    hipStream_t s = m->stream;
    size_t n1 = static_cast<size_t>(m->N) + 1;
    if (owner_start) LF_HIP(hipMemcpyAsync(owner_start, m->owner_start, 4 * n1, hipMemcpyDeviceToHost, s));
    if (losort && m->F) LF_HIP(hipMemcpyAsync(losort, m->losort, 4 * static_cast<size_t>(m->F), hipMemcpyDeviceToHost, s));
    if (losort_start) LF_HIP(hipMemcpyAsync(losort_start, m->losort_start, 4 * n1, hipMemcpyDeviceToHost, s));
    if (bface_start) LF_HIP(hipMemcpyAsync(bface_start, m->bface_start, 4 * n1, hipMemcpyDeviceToHost, s));
    if (bface_list && m->B) LF_HIP(hipMemcpyAsync(bface_list, m->bface_list, 4 * static_cast<size_t>(m->B), hipMemcpyDeviceToHost, s));
    LF_HIP(hipStreamSynchronize(s));
    return LF_OK;
}

}  // extern "C"
