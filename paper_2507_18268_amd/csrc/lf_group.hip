// Grouped stepping of several precision-form problems (the C ABI's lf_group_*).
//
// Each member runs the precision form's step exactly as lf_step does (the same
// kernels in the same order on its own data); what the group changes is who
// launches them.  The inner FP32 iterations of all members that are iterating
// go out as one launch per kernel on the group's stream (each member keeps its
// own workgroups, rows and partial sums, so its arithmetic is unchanged); the
// assembly with the start of the solve, and the turn from one refinement pass
// to the next, go to the member's own stream.  The streams are ordered by
// events: a member's stream waits for the group block that last touched it,
// and the group waits for a member's own work before the member's next block.
// After each block of inner iterations the members' solver states are
// gathered into one array and copied to the host, where each member's next
// move is decided: keep iterating, turn to the next pass (no-ops if the solve
// has finished), or finish the step (statistics, snapshot of T, next step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lf_solver.h"

namespace lf {

struct GroupMember {
    lf_problem *P = nullptr;
    int32_t n_steps = 0, step = 0;
    double *snap = nullptr;
    lf_solve_stats *stats = nullptr;
    enum Stage { kFree, kIterating, kFinishing } stage = kFree;
    bool wait = false;          // the group stream waits on ev before the member's next block
    hipEvent_t ev = nullptr;    // recorded on the member's stream after its own work
    int64_t launched = 0;       // inner iterations launched in the current step
};

// a member's field between solver and mesh order (a copy when the mesh keeps its order)
__global__ void k_grp_to_mesh(int32_t n, const int32_t *__restrict__ iperm, const double *__restrict__ x,
                              double *__restrict__ y) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) y[iperm[r]] = x[r];
}
__global__ void k_grp_to_solver(int32_t n, const int32_t *__restrict__ iperm, const double *__restrict__ x,
                                double *__restrict__ y) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) y[r] = x[iperm[r]];
}

}  // namespace lf

struct lf_group {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t max_members = 0, iters = 2;
    lf::InnerMember *d_tab = nullptr, *h_tab = nullptr;
    lf::PcgState *d_states = nullptr, *h_states = nullptr;
    std::vector<lf::GroupMember> members;
    hipEvent_t ev_block = nullptr;
    bool in_flight = false;
    lf::GroupLaunch last{};
    std::vector<lf_problem *> done;     // finished runs not yet handed back
};

using namespace lf;

namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

size_t group_bytes(int32_t max_members) {
    return align256(sizeof(InnerMember) * static_cast<size_t>(max_members)) +
           align256(sizeof(PcgState) * static_cast<size_t>(max_members));
}

lf_status check_member(const lf_group *g, const lf_problem *P) {
    if (P->opts.precision != LF_PREC_MIXED) { set_error("a group runs LF_PREC_MIXED problems"); return LF_EINVAL; }
    if (P->opts.precond != LF_PC_DIAGONAL) { set_error("a group runs the diagonal preconditioner"); return LF_EINVAL; }
    if (P->nonorth) { set_error("a group runs orthogonal meshes (no corrector loop)"); return LF_EINVAL; }
    if (P->walk || P->box || P->rb) {
        set_error("a group runs the one-row-per-thread products (lf_problem_amul_walk 0)");
        return LF_EINVAL;
    }
    if (P->mesh->device != g->device) {
        set_error("the problem lives on device %d, the group on %d", P->mesh->device, g->device);
        return LF_EINVAL;
    }
    if (P->sp.grid_mx_amul != P->sp.grid_mx) { set_error("unexpected product grid"); return LF_EINVAL; }
    return LF_OK;
}

// enqueue a member's next step on its own stream (after the group's last block)
lf_status start_step(lf_group *g, GroupMember &m, bool after_block) {
    lf_problem *P = m.P;
    if (after_block) LF_HIP(hipStreamWaitEvent(P->stream, g->ev_block, 0));
    LF_TRY(mixed_enqueue_step_start(P, P->stream));
    P->assembled = true;
    P->scaled32 = true;
    LF_HIP(hipEventRecord(m.ev, P->stream));
    m.wait = true;
    m.launched = 0;
    m.stage = GroupMember::kIterating;
    return LF_OK;
}

// the member's step has ended (state h): its stats, the snapshot of T, then
// the next step or the end of its run
lf_status finish_step(lf_group *g, GroupMember &m, const PcgState &h) {
    lf_problem *P = m.P;
    if (m.stats) {
        lf_solve_stats &o = m.stats[m.step];
        std::memset(&o, 0, sizeof(o));
        o.initial_residual = h.res0;
        o.final_residual = h.res;
        o.n_iter = h.n_iter;
        o.converged = h.converged;
        o.nonfinite = h.nonfinite;
        o.n_outer = h.n_outer;
    }
    P->last_iters = h.n_iter;
    P->last_outer = h.n_outer;
    LF_HIP(hipStreamWaitEvent(P->stream, g->ev_block, 0));
    if (m.snap) {
        const lf_mesh *msh = P->mesh;
        double *dst = m.snap + static_cast<int64_t>(m.step) * msh->N;
        if (msh->iperm)
            hipLaunchKernelGGL(k_grp_to_mesh, dim3((msh->N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream,
                               msh->N, msh->iperm, P->T, dst);
        else
            LF_HIP(hipMemcpyAsync(dst, P->T, sizeof(double) * msh->N, hipMemcpyDeviceToDevice, P->stream));
        LF_HIP(hipGetLastError());
    }
    ++m.step;
    if (!h.nonfinite && m.step < m.n_steps) return start_step(g, m, false);
    LF_HIP(hipEventRecord(m.ev, P->stream));
    m.stage = GroupMember::kFinishing;
    return LF_OK;
}

// the result of the block that just finished
lf_status consume_block(lf_group *g) {
    for (int32_t i = 0; i < g->last.n; ++i) {
        GroupMember &m = g->members[g->last.slot[i]];
        const PcgState &h = g->h_states[g->last.slot[i]];
        m.launched += g->iters;
        if (h.done) {
            LF_TRY(finish_step(g, m, h));
        } else if (m.launched > 4 * (static_cast<int64_t>(m.P->sp.max_iter) + 8) + 64 * m.P->sp.max_outer) {
            set_error("a member never reached the end of its solve after %lld inner iterations",
                      static_cast<long long>(m.launched));
            return LF_ESTATE;
        } else if (h.inner_done) {
            // the pass has ended: its end and the next pass's start on the
            // member's stream (no-ops if the outer check finishes the solve)
            lf_problem *P = m.P;
            LF_HIP(hipStreamWaitEvent(P->stream, g->ev_block, 0));
            LF_TRY(mixed_enqueue_pass_turn(P, P->stream));
            LF_HIP(hipEventRecord(m.ev, P->stream));
            m.wait = true;
        }
    }
    return LF_OK;
}

// the next block: iters inner iterations of every iterating member, then the
// gather of their states
lf_status launch_block(lf_group *g) {
    GroupLaunch gl{};
    int64_t blocks = 0;
    for (int32_t s = 0; s < g->max_members; ++s) {
        const GroupMember &m = g->members[s];
        if (m.stage != GroupMember::kIterating) continue;
        gl.slot[gl.n] = s;
        gl.begin[gl.n] = static_cast<int32_t>(blocks);
        blocks += m.P->sp.grid_mx;
        ++gl.n;
    }
    if (gl.n == 0) return LF_OK;
    if (blocks > INT32_MAX) { set_error("group launch too large"); return LF_EINVAL; }
    gl.begin[gl.n] = static_cast<int32_t>(blocks);
    for (int32_t i = 0; i < gl.n; ++i) {
        GroupMember &m = g->members[gl.slot[i]];
        if (m.wait) {
            LF_HIP(hipStreamWaitEvent(g->stream, m.ev, 0));
            m.wait = false;
        }
    }
    for (int32_t k = 0; k < g->iters; ++k) launch_group_iteration(g->d_tab, gl, g->stream);
    launch_group_gather(g->d_tab, gl, g->d_states, g->stream);
    LF_HIP(hipGetLastError());
    LF_HIP(hipMemcpyAsync(g->h_states, g->d_states, sizeof(PcgState) * static_cast<size_t>(g->max_members),
                          hipMemcpyDeviceToHost, g->stream));
    LF_HIP(hipEventRecord(g->ev_block, g->stream));
    g->in_flight = true;
    g->last = gl;
    return LF_OK;
}

void release(lf_group *g) {
    for (auto &m : g->members)
        if (m.ev) (void)hipEventDestroy(m.ev);
    if (g->ev_block) (void)hipEventDestroy(g->ev_block);
    if (g->h_tab) (void)hipHostFree(g->h_tab);
    if (g->h_states) (void)hipHostFree(g->h_states);
    delete g;
}

}  // namespace

extern "C" {

size_t lf_group_workspace_bytes(int32_t max_members) {
    if (max_members < 1 || max_members > kGroupMax) return 0;
    return group_bytes(max_members);
}

lf_status lf_group_create(int32_t max_members, int32_t iters_per_block, void *ws, size_t ws_bytes, void *stream,
                          lf_group **out) {
    clear_error();
    if (!out || !ws) { set_error("NULL argument"); return LF_EINVAL; }
    *out = nullptr;
    if (max_members < 1 || max_members > kGroupMax) {
        set_error("max_members must be in [1, %d]", kGroupMax);
        return LF_EINVAL;
    }
    if (iters_per_block < 0 || iters_per_block > 64) { set_error("iters_per_block must be in [0, 64]"); return LF_EINVAL; }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) { set_error("workspace must be 256-byte aligned"); return LF_EINVAL; }
    if (ws_bytes < group_bytes(max_members)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, group_bytes(max_members));
        return LF_EINVAL;
    }
    lf_group *g = new (std::nothrow) lf_group();
    if (!g) { set_error("host allocation failed"); return LF_ENOMEM; }
    g->max_members = max_members;
    g->iters = iters_per_block > 0 ? iters_per_block : 2;
    g->stream = static_cast<hipStream_t>(stream);
    g->members.resize(static_cast<size_t>(max_members));
    char *base = static_cast<char *>(ws);
    g->d_tab = reinterpret_cast<InnerMember *>(base);
    g->d_states = reinterpret_cast<PcgState *>(base + align256(sizeof(InnerMember) * max_members));
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&g->h_tab), sizeof(InnerMember) * max_members,
                                           hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&g->h_states), sizeof(PcgState) * max_members,
                                           hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_block, hipEventDisableTiming);
    for (auto &m : g->members)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m.ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        set_error("group set-up failed: %s", hipGetErrorString(e));
        release(g);
        return LF_EDEVICE;
    }
    std::memset(g->h_states, 0, sizeof(PcgState) * max_members);
    *out = g;
    return LF_OK;
}

lf_status lf_group_destroy(lf_group *g) {
    clear_error();
    if (!g) return LF_OK;
    for (const auto &m : g->members)
        if (m.stage != GroupMember::kFree) { set_error("members are still running"); return LF_ESTATE; }
    if (!g->done.empty()) { set_error("finished members not handed back yet (lf_group_poll)"); return LF_ESTATE; }
    if (g->in_flight) (void)hipEventSynchronize(g->ev_block);
    release(g);
    return LF_OK;
}

lf_status lf_group_add(lf_group *g, lf_problem *P, int32_t n_steps, const double *T0, double *snapshots,
                       lf_solve_stats *stats) {
    clear_error();
    if (!g || !P || n_steps < 1) { set_error("bad argument"); return LF_EINVAL; }
    if (problem_in_flight(P)) { set_error("the problem runs already"); return LF_ESTATE; }
    LF_TRY(check_member(g, P));
    int32_t slot = -1;
    for (int32_t s = 0; s < g->max_members && slot < 0; ++s)
        if (g->members[s].stage == GroupMember::kFree) slot = s;
    if (slot < 0) { set_error("the group is full (%d members)", g->max_members); return LF_EBUDGET; }
    GroupMember &m = g->members[slot];
    if (T0) {
        // the starting field, on the member's stream before its first step
        const lf_mesh *msh = P->mesh;
        if (msh->iperm)
            hipLaunchKernelGGL(k_grp_to_solver, dim3((msh->N + kBlock - 1) / kBlock), dim3(kBlock), 0, P->stream,
                               msh->N, msh->iperm, T0, P->T);
        else
            LF_HIP(hipMemcpyAsync(P->T, T0, sizeof(double) * msh->N, hipMemcpyDeviceToDevice, P->stream));
        LF_HIP(hipGetLastError());
    }
    // the descriptor, ordered on the group's stream before any block reads it
    g->h_tab[slot] = inner_member(P);
    LF_HIP(hipMemcpyAsync(g->d_tab + slot, g->h_tab + slot, sizeof(InnerMember), hipMemcpyHostToDevice, g->stream));
    m.P = P;
    m.n_steps = n_steps;
    m.step = 0;
    m.snap = snapshots;
    m.stats = stats;
    P->group = g;
    const lf_status st = start_step(g, m, false);
    if (st != LF_OK) {
        P->group = nullptr;
        m.P = nullptr;
        m.stage = GroupMember::kFree;
        m.wait = false;
    }
    return st;
}

lf_status lf_group_poll(lf_group *g, lf_problem **finished, int32_t max_finished, int32_t *n_finished,
                        int32_t *n_active) {
    clear_error();
    if (!g || !n_finished || !n_active || max_finished < 0 || (max_finished > 0 && !finished)) {
        set_error("bad argument");
        return LF_EINVAL;
    }
    *n_finished = 0;
    if (g->in_flight) {
        const hipError_t q = hipEventQuery(g->ev_block);
        if (q == hipSuccess) {
            g->in_flight = false;
            LF_TRY(consume_block(g));
        } else if (q != hipErrorNotReady) {
            set_error("hipEventQuery failed: %s", hipGetErrorString(q));
            return LF_EDEVICE;
        }
    }
    // runs whose last snapshot has been written
    for (auto &m : g->members) {
        if (m.stage != GroupMember::kFinishing) continue;
        const hipError_t q = hipEventQuery(m.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) { set_error("hipEventQuery failed: %s", hipGetErrorString(q)); return LF_EDEVICE; }
        m.P->group = nullptr;
        g->done.push_back(m.P);
        m.P = nullptr;
        m.stage = GroupMember::kFree;
    }
    if (!g->in_flight) LF_TRY(launch_block(g));
    const int32_t k = static_cast<int32_t>(std::min<size_t>(g->done.size(), static_cast<size_t>(max_finished)));
    for (int32_t i = 0; i < k; ++i) finished[i] = g->done[static_cast<size_t>(i)];
    g->done.erase(g->done.begin(), g->done.begin() + k);
    *n_finished = k;
    int32_t active = static_cast<int32_t>(g->done.size());
    for (const auto &m : g->members) active += m.stage != GroupMember::kFree;
    *n_active = active;
    return LF_OK;
}

}  // extern "C"
