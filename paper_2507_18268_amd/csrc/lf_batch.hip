// Batched form: one persistent kernel over a task table of independent
// problems (mesh, DT, dt, boundary conditions, T).
//
// Each workgroup takes the next task from the table (an integer counter) and
// runs all of its time steps alone: assembly in FP64 with an FP32 copy of
// the coefficients, then the precision form's refinement (FP64 true residual
// and update, FP32 inner PCG with FP64 dot products, alpha and beta).  Phases
// are separated by workgroup barriers only; no workgroup ever waits for
// another, so the grid always drains.  Every sum runs in a fixed order inside
// the workgroup, so a problem's result does not depend on which other
// problems share the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "lf_solver.h"

namespace lf {

struct BatchTask {
    // mesh (sliced row layout and geometry)
    const int32_t *soff, *scol, *sface;
    const uint8_t *rlen;
    const double *V, *mag_sf, *delta;
    const double *emag_sf, *edelta;   // per entry of the row layout, or null
    const int32_t *bface_start, *bface_list, *bface_patch;
    const double *bmag_sf, *bdelta;
    const int32_t *patch_type;
    const double *patch_value;
    // problem
    double *T, *coef, *diagB, *srcB, *r;
    float *coef32, *diag32, *rD32, *r32, *p32, *q32, *d32;
    double *snap;          // [n_steps][n] copies of T after each step (mesh cell order), or null
    const int32_t *iperm;  // mesh cell of each solver row, or null (same order)
    // band layout of the problem's coefficients (nb = 3; 0: sliced row layout)
    const double *band_mag_sf, *band_delta;
    int32_t nb, band_d[kMaxBands];
    double DT, dt, tol, rel_tol, inner_tol;
    int32_t n, max_iter, max_outer, pad;
};

// tightening of the refinement target, as in the single-problem precision form
constexpr double kBatchTighten = 0.1;

template <int BS>
__device__ __forceinline__ double bsum1(double v) {
    double a[1] = {v};
    block_sum<BS, 1>(a);
    return a[0];
}

template <int BS>
__device__ __forceinline__ void bsum2(double &a0, double &a1) {
    double a[2] = {a0, a1};
    block_sum<BS, 2>(a);
    a0 = a[0];
    a1 = a[1];
}

// The task's arrays are distinct allocations: taking them into __restrict__
// locals lets the compiler overlap the loads of several rows of a loop.
template <int BS, class Lay>
__device__ void solve_task(const BatchTask &tk, const Lay &L, int32_t n_steps, lf_solve_stats *__restrict__ stats) {
    const int32_t n = tk.n;
    const double *__restrict__ V = tk.V;
    const int32_t *__restrict__ bface_start = tk.bface_start;
    const int32_t *__restrict__ bface_list = tk.bface_list;
    const int32_t *__restrict__ bface_patch = tk.bface_patch;
    const double *__restrict__ bmag_sf = tk.bmag_sf;
    const double *__restrict__ bdelta = tk.bdelta;
    const int32_t *__restrict__ patch_type = tk.patch_type;
    const double *__restrict__ patch_value = tk.patch_value;
    double *__restrict__ T = tk.T;
    double *__restrict__ coef = tk.coef;
    double *__restrict__ diagB = tk.diagB;
    double *__restrict__ srcB = tk.srcB;
    double *__restrict__ r = tk.r;
    float *__restrict__ coef32 = tk.coef32;
    float *__restrict__ diag32 = tk.diag32;
    float *__restrict__ rD32 = tk.rD32;
    float *__restrict__ r32 = tk.r32;
    float *__restrict__ p32 = tk.p32;
    float *__restrict__ q32 = tk.q32;
    float *__restrict__ d32 = tk.d32;
    const int32_t tid = static_cast<int32_t>(threadIdx.x);
    const double rdt = 1.0 / tk.dt;
    const double DT = tk.DT;
    for (int32_t step = 0; step < n_steps; ++step) {
        // ---- mean of x0 = T
        double sx = 0.0;
        for (int32_t c = tid; c < n; c += BS) sx += T[c];
        const double x_avg = bsum1<BS>(sx) / static_cast<double>(n);
        // ---- assembly (FP64 + FP32 copy), r0 = b - A x0, normalisation terms
        double a_r = 0.0, a_nf = 0.0;
        for (int32_t c = tid; c < n; c += BS) {
            RowCoefs<Lay> rcf;
            const double lap_diag = assemble_coefs<false>(L, c, DT, coef, nullptr, rcf);
            store_coef32(L, c, coef, rcf, coef32);
            const double v = V[c];
            const double xc = T[c];
            double db = rdt * v - lap_diag;
            double sb = (rdt * xc) * v;
            for (int32_t i = bface_start[c]; i < bface_start[c + 1]; ++i) {
                const int32_t b = bface_list[i];
                const int32_t pt = bface_patch[b];
                if (patch_type[pt] == LF_BC_FIXED_VALUE) {
                    const double g = DT * bmag_sf[b];
                    db += g * bdelta[b];
                    sb += g * (bdelta[b] * patch_value[pt]);
                }
            }
            diagB[c] = db;
            srcB[c] = sb;
            diag32[c] = static_cast<float>(db);
            rD32[c] = static_cast<float>(1.0 / db);
            double ax = db * xc, sa = db;
            row_amul_sum(L, c, coef, rcf, T, ax, sa);
            const double rc = sb - ax;
            r[c] = rc;
            const double pa = sa * x_avg;
            a_r += fabs(rc);
            a_nf += fabs(ax - pa) + fabs(sb - pa);
        }
        bsum2<BS>(a_r, a_nf);
        const double nf = a_nf + 1e-20;
        const double res0 = a_r / nf;
        double res = res0;
        int32_t n_iter = 0, n_outer = 0;
        bool nonfinite = !isfinite(res0);
        bool conv = check_conv(res0, res0, tk.tol, tk.rel_tol);
        bool tight = check_conv(res0, res0, kBatchTighten * tk.tol, kBatchTighten * tk.rel_tol);
        // ---- refinement passes
        while (!nonfinite && !tight && n_outer < tk.max_outer && n_iter < tk.max_iter) {
            double s_r = 0.0, s_wr = 0.0;
            #pragma unroll 2
            for (int32_t c = tid; c < n; c += BS) {
                const float rc = static_cast<float>(r[c]);
                r32[c] = rc;
                d32[c] = 0.0f;
                const float wc = rD32[c] * rc;
                s_r += fabs(static_cast<double>(rc));
                s_wr += static_cast<double>(wc) * static_cast<double>(rc);
            }
            bsum2<BS>(s_r, s_wr);
            const double target = fmax(tk.inner_tol * s_r, 0.5 * kBatchTighten * tk.tol * nf);
            double wArA = s_wr;
            double beta = 0.0;
            bool inner_done = (s_r <= target) || !(s_wr > 0.0);
            int32_t inner_iter = 0;
            while (!inner_done) {
                const float fb = static_cast<float>(beta);
                #pragma unroll 2
                for (int32_t c = tid; c < n; c += BS) {
                    const float wc = rD32[c] * r32[c];
                    p32[c] = inner_iter == 0 ? wc : wc + fb * p32[c];
                }
                __syncthreads();
                double s_pq = 0.0;
                for (int32_t c = tid; c < n; c += BS) {
                    const float pc = p32[c];
                    const float qc = layout_dot(L, c, coef32, p32, diag32[c] * pc);
                    q32[c] = qc;
                    s_pq += static_cast<double>(qc) * static_cast<double>(pc);
                }
                const double pq = bsum1<BS>(s_pq);
                if (!isfinite(pq)) { nonfinite = true; break; }
                if (!(fabs(pq) > 0.0)) break;
                const double alpha = wArA / pq;
                const float fa = static_cast<float>(alpha);
                double u_r = 0.0, u_wr = 0.0;
                #pragma unroll 2
                for (int32_t c = tid; c < n; c += BS) {
                    d32[c] += fa * p32[c];
                    const float rc = r32[c] - fa * q32[c];
                    r32[c] = rc;
                    const float wc = rD32[c] * rc;
                    u_r += fabs(static_cast<double>(rc));
                    u_wr += static_cast<double>(wc) * static_cast<double>(rc);
                }
                bsum2<BS>(u_r, u_wr);
                ++inner_iter;
                ++n_iter;
                if (!isfinite(u_r) || !isfinite(u_wr)) { nonfinite = true; break; }
                if (u_r <= target || n_iter >= tk.max_iter || !(u_wr > 0.0)) {
                    inner_done = true;
                } else {
                    beta = u_wr / wArA;
                    wArA = u_wr;
                }
            }
            if (nonfinite) break;
            // T += d, then the FP64 true residual
            #pragma unroll 2
            for (int32_t c = tid; c < n; c += BS) T[c] += static_cast<double>(d32[c]);
            __syncthreads();
            double o_r = 0.0;
            for (int32_t c = tid; c < n; c += BS) {
                const double ax = layout_dot(L, c, coef, T, diagB[c] * T[c]);
                const double rc = srcB[c] - ax;
                r[c] = rc;
                o_r += fabs(rc);
            }
            o_r = bsum1<BS>(o_r);
            res = o_r / nf;
            ++n_outer;
            nonfinite = !isfinite(res);
            conv = check_conv(res, res0, tk.tol, tk.rel_tol);
            tight = check_conv(res, res0, kBatchTighten * tk.tol, kBatchTighten * tk.rel_tol);
        }
        if (tk.snap) {
            double *__restrict__ out = tk.snap + static_cast<int64_t>(step) * n;
            const int32_t *__restrict__ ip = tk.iperm;
            #pragma unroll 2
            for (int32_t c = tid; c < n; c += BS) out[ip ? ip[c] : c] = T[c];
        }
        if (tid == 0) {
            lf_solve_stats st;
            st.initial_residual = res0;
            st.final_residual = res;
            st.n_iter = n_iter;
            st.converged = conv ? 1 : 0;
            st.singular = 0;
            st.nonfinite = nonfinite ? 1 : 0;
            st.n_outer = n_outer;
            st.reserved = 0;
            st.assemble_ms = 0.0;
            st.solve_ms = 0.0;
            stats[step] = st;
        }
        __syncthreads();
        if (nonfinite) {
            for (int32_t s2 = step + 1 + tid; s2 < n_steps; s2 += BS) {
                lf_solve_stats st{};
                st.nonfinite = 1;
                stats[s2] = st;
            }
            return;
        }
    }
}

template <int BS>
__global__ void __launch_bounds__(BS) k_batch(const BatchTask *__restrict__ tasks, int32_t n_tasks,
                                             int32_t *__restrict__ counter, int32_t n_steps,
                                             lf_solve_stats *__restrict__ stats) {
    __shared__ int32_t s_task;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t t = s_task;
        __syncthreads();
        if (t >= n_tasks) return;
        const BatchTask &tk = tasks[t];
        lf_solve_stats *st = stats + static_cast<int64_t>(t) * n_steps;
        if (tk.nb == 3) {
            BandLayout<3> L;
            L.n = tk.n;
#pragma unroll
            for (int k = 0; k < 3; ++k) L.d[k] = tk.band_d[k];
            L.mag_sf = tk.band_mag_sf;
            L.delta = tk.band_delta;
            solve_task<BS>(tk, L, n_steps, st);
        } else {
            const SellLayout L{MeshRows{tk.soff, tk.scol, tk.sface, tk.rlen}, tk.mag_sf, tk.delta, tk.emag_sf,
                               tk.edelta};
            solve_task<BS>(tk, L, n_steps, st);
        }
    }
}

__global__ void k_zero_counter(int32_t *counter) { *counter = 0; }

}  // namespace lf

using namespace lf;

struct lf_batch {
    int32_t max_tasks = 0, max_steps = 0;
    hipStream_t stream = nullptr;
    BatchTask *d_tasks = nullptr;
    int32_t *d_counter = nullptr;
    lf_solve_stats *d_stats = nullptr;
    BatchTask *h_tasks = nullptr;          // pinned staging of the task table
    lf_solve_stats *h_stats = nullptr;     // pinned
    hipEvent_t done = nullptr, start = nullptr;
    int32_t last_n = 0, last_steps = 0;
    bool in_flight = false;
    int device = 0;
};

static void carve_batch(Carver &cv, int32_t max_tasks, int32_t max_steps, lf_batch *b) {
    auto *tasks = cv.take<BatchTask>(static_cast<size_t>(max_tasks));
    auto *counter = cv.take<int32_t>(1);
    auto *stats = cv.take<lf_solve_stats>(static_cast<size_t>(max_tasks) * max_steps);
    if (b) {
        b->d_tasks = tasks;
        b->d_counter = counter;
        b->d_stats = stats;
    }
}

extern "C" {

size_t lf_batch_workspace_bytes(int32_t max_tasks, int32_t max_steps) {
    if (max_tasks < 1 || max_steps < 1) return 0;
    Carver cv(nullptr);
    carve_batch(cv, max_tasks, max_steps, nullptr);
    return cv.bytes();
}

lf_status lf_batch_create(int32_t max_tasks, int32_t max_steps, void *ws, size_t ws_bytes, void *stream,
                          lf_batch **out) {
    clear_error();
    if (!out || max_tasks < 1 || max_steps < 1) { set_error("bad argument"); return LF_EINVAL; }
    *out = nullptr;
    Carver dry(nullptr);
    carve_batch(dry, max_tasks, max_steps, nullptr);
    if (!ws || ws_bytes < dry.bytes() || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
        set_error("batch workspace too small or misaligned: need %zu bytes, 256-aligned", dry.bytes());
        return LF_ENOMEM;
    }
    lf_batch *b = new (std::nothrow) lf_batch();
    if (!b) { set_error("host allocation failed"); return LF_ENOMEM; }
    b->max_tasks = max_tasks;
    b->max_steps = max_steps;
    b->stream = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    carve_batch(cv, max_tasks, max_steps, b);
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&b->h_tasks), sizeof(BatchTask) * max_tasks, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&b->h_stats),
                          sizeof(lf_solve_stats) * static_cast<size_t>(max_tasks) * max_steps, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&b->done);
    if (e == hipSuccess) e = hipEventCreate(&b->start);
    if (e != hipSuccess) {
        set_error("batch setup failed: %s", hipGetErrorString(e));
        lf_batch_destroy(b);
        return LF_EDEVICE;
    }
    *out = b;
    return LF_OK;
}

lf_status lf_batch_destroy(lf_batch *b) {
    if (!b) return LF_OK;
    if (b->in_flight && b->done) (void)hipEventSynchronize(b->done);
    if (b->h_tasks) (void)hipHostFree(b->h_tasks);
    if (b->h_stats) (void)hipHostFree(b->h_stats);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
    return LF_OK;
}

lf_status lf_batch_launch(lf_batch *b, int32_t n, lf_problem *const *problems, double *const *snapshots,
                          int32_t n_steps, int32_t block_threads, int32_t n_workgroups) {
    clear_error();
    if (!b || n < 1 || !problems || n_steps < 1) { set_error("bad argument"); return LF_EINVAL; }
    if (n > b->max_tasks || n_steps > b->max_steps) {
        set_error("batch holds at most %d tasks x %d steps", b->max_tasks, b->max_steps);
        return LF_EINVAL;
    }
    if (b->in_flight) { set_error("previous launch not finished (lf_batch_wait / lf_batch_poll)"); return LF_ESTATE; }
    if (block_threads != 256 && block_threads != 512 && block_threads != 1024) {
        set_error("block_threads must be 256, 512 or 1024");
        return LF_EINVAL;
    }
    {
        std::vector<const lf_problem *> seen(problems, problems + n);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) {
            set_error("a problem is listed twice (each task writes its problem's T and vectors)");
            return LF_EINVAL;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        const lf_problem *P = problems[i];
        if (!P) { set_error("problem %d is NULL", i); return LF_EINVAL; }
        if (problem_in_flight(P)) { set_error("problem %d: an lf_step_begin run is in flight", i); return LF_ESTATE; }
        if (P->opts.precision != LF_PREC_MIXED || P->opts.precond != LF_PC_DIAGONAL) {
            set_error("problem %d: the batched form needs LF_PREC_MIXED with the diagonal preconditioner", i);
            return LF_EINVAL;
        }
        if (P->mesh->device != b->device) { set_error("problem %d lives on another device", i); return LF_EINVAL; }
        if (P->nonorth) {
            set_error("problem %d: the batched kernel has no non-orthogonal correction", i);
            return LF_EINVAL;
        }
        const lf_mesh *m = P->mesh;
        BatchTask &t = b->h_tasks[i];
        t.soff = m->soff; t.scol = m->scol; t.sface = m->sface; t.rlen = m->rlen;
        t.V = m->V; t.mag_sf = m->mag_sf; t.delta = m->delta;
        t.emag_sf = m->emag_sf; t.edelta = m->edelta;
        t.bface_start = m->rbface_start; t.bface_list = m->rbface_list; t.bface_patch = m->bface_patch;
        t.iperm = m->iperm;
        t.bmag_sf = m->bmag_sf; t.bdelta = m->bdelta;
        t.patch_type = P->patch_type; t.patch_value = P->patch_value;
        t.T = P->T; t.coef = P->coef; t.diagB = P->diagB; t.srcB = P->srcB; t.r = P->r;
        t.coef32 = P->coef32; t.diag32 = P->diag32; t.rD32 = P->rD32; t.r32 = P->r32;
        t.p32 = P->p32; t.q32 = P->q32; t.d32 = P->d32;
        t.snap = snapshots ? snapshots[i] : nullptr;
        if (P->banded && m->n_bands != 3) {
            set_error("problem %d: the batched form takes the band layout of 3-band (structured 3-D) meshes "
                      "only; create it with LF_LAYOUT_ROWS", i);
            return LF_EINVAL;
        }
        t.nb = P->banded ? 3 : 0;
        for (int k = 0; k < kMaxBands; ++k) t.band_d[k] = k < m->n_bands ? m->band_d[k] : 0;
        t.band_mag_sf = m->band_mag_sf;
        t.band_delta = m->band_delta;
        t.DT = P->DT; t.dt = P->dt; t.tol = P->sp.tol; t.rel_tol = P->sp.rel_tol; t.inner_tol = P->sp.inner_tol;
        t.n = m->N; t.max_iter = P->sp.max_iter; t.max_outer = P->sp.max_outer; t.pad = 0;
    }
    hipStream_t s = b->stream;
    int32_t g = n_workgroups > 0 ? std::min(n_workgroups, n) : n;
    LF_HIP(hipMemcpyAsync(b->d_tasks, b->h_tasks, sizeof(BatchTask) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, b->d_counter);
    LF_HIP(hipEventRecord(b->start, s));
    switch (block_threads) {
        case 256: hipLaunchKernelGGL(k_batch<256>, dim3(g), dim3(256), 0, s, b->d_tasks, n, b->d_counter, n_steps, b->d_stats); break;
        case 512: hipLaunchKernelGGL(k_batch<512>, dim3(g), dim3(512), 0, s, b->d_tasks, n, b->d_counter, n_steps, b->d_stats); break;
        default: hipLaunchKernelGGL(k_batch<1024>, dim3(g), dim3(1024), 0, s, b->d_tasks, n, b->d_counter, n_steps, b->d_stats); break;
    }
    LF_HIP(hipGetLastError());
    LF_HIP(hipMemcpyAsync(b->h_stats, b->d_stats, sizeof(lf_solve_stats) * static_cast<size_t>(n) * n_steps,
                          hipMemcpyDeviceToHost, s));
    LF_HIP(hipEventRecord(b->done, s));
    b->last_n = n;
    b->last_steps = n_steps;
    b->in_flight = true;
    return LF_OK;
}

lf_status lf_batch_poll(lf_batch *b, int32_t *finished) {
    clear_error();
    if (!b || !finished) { set_error("bad argument"); return LF_EINVAL; }
    if (!b->in_flight) { *finished = 1; return LF_OK; }
    hipError_t e = hipEventQuery(b->done);
    if (e == hipSuccess) { *finished = 1; b->in_flight = false; return LF_OK; }
    if (e == hipErrorNotReady) { *finished = 0; return LF_OK; }
    set_error("hipEventQuery failed: %s", hipGetErrorString(e));
    return LF_EDEVICE;
}

lf_status lf_batch_wait(lf_batch *b) {
    clear_error();
    if (!b) { set_error("bad argument"); return LF_EINVAL; }
    if (!b->in_flight) return LF_OK;
    LF_HIP(hipEventSynchronize(b->done));
    b->in_flight = false;
    return LF_OK;
}

lf_status lf_batch_stats(lf_batch *b, lf_solve_stats *stats, double *elapsed_ms) {
    clear_error();
    if (!b) { set_error("bad argument"); return LF_EINVAL; }
    if (b->in_flight) { set_error("launch still running"); return LF_ESTATE; }
    if (stats) std::memcpy(stats, b->h_stats, sizeof(lf_solve_stats) * static_cast<size_t>(b->last_n) * b->last_steps);
    if (elapsed_ms) {
        float ms = 0.f;
        LF_HIP(hipEventElapsedTime(&ms, b->start, b->done));
        *elapsed_ms = ms;
    }
    return LF_OK;
}

}  // extern "C"
