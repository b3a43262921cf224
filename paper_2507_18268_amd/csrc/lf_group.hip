// Grouped stepping of several precision-form problems (the C ABI's lf_group_*).
//
// Each member runs the precision form's step exactly as lf_step does (the same
// kernel bodies in the same order on its own data, with its own workgroups
// and fixed-order partial sums); what the group changes is who launches them.
// Every launch serves all members that need that kernel at that point, on the
// group's stream: copies (T0 in, snapshots out), the start of a step (x0
// sums, mean, assembly fused with the start of the solve, FP32 scaling,
// initial decision, start of the first refinement pass), the turn from one
// refinement pass to the next (correction, FP64 residual, outer check, start
// of the next pass: no-ops once the solve is done), then a block of inner FP32
// iterations of every iterating member, and the gather of the members' solver
// states into one array copied to the host.  From those states the host
// decides each member's next move: keep iterating, turn to the next pass, or
// finish the step (statistics, snapshot of T, next step or end of the run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lf_solver.h"

namespace lf {

struct GroupMember {
    lf_problem *P = nullptr;        // null: free slot
    int32_t n_steps = 0, step = 0;
    double *snap = nullptr;
    lf_solve_stats *stats = nullptr;
    const double *T0 = nullptr;     // copied in by the next launch
    bool start = false;             // the next launch starts step `step`
    bool turn = false;              // the next launch turns to the next refinement pass
    int32_t snap_step = -1;         // the next launch copies T into this step's snapshot
    bool final = false;             // the run ends once final_launch has completed
    int64_t final_launch = -1;
    int64_t launched = 0;           // inner iterations launched in the current step
};

// copies of several members' fields in one launch: entry i moves cells[i]
// values, its workgroups from begin[i]; mode 0 plain, 1 into mesh order
// (y[perm[r]] = x[r]), 2 into solver order (y[r] = x[perm[r]])
struct GroupCopy {
    int32_t n;
    int32_t cells[kGroupMax];
    int32_t mode[kGroupMax];
    const double *src[kGroupMax];
    double *dst[kGroupMax];
    const int32_t *perm[kGroupMax];
    int32_t begin[kGroupMax + 1];
};

__global__ void __launch_bounds__(kBlock) k_grp_copy(GroupCopy gc) {
    const int32_t b = static_cast<int32_t>(blockIdx.x);
    int32_t i = 0;
    while (i + 1 < gc.n && b >= gc.begin[i + 1]) ++i;
    const int64_t r = static_cast<int64_t>(b - gc.begin[i]) * kBlock + threadIdx.x;
    if (r >= gc.cells[i]) return;
    const double *x = gc.src[i];
    double *y = gc.dst[i];
    if (gc.mode[i] == 0) y[r] = x[r];
    else if (gc.mode[i] == 1) y[gc.perm[i][r]] = x[r];
    else y[r] = x[gc.perm[i][r]];
}

}  // namespace lf

struct lf_group {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t max_members = 0, iters = 2;
    lf::MemberDesc *d_tab = nullptr, *h_tab = nullptr;
    lf::PcgState *d_states = nullptr, *h_states = nullptr;
    std::vector<lf::GroupMember> members;
    hipEvent_t ev_block = nullptr;
    bool in_flight = false;
    int64_t launches = 0;           // launches enqueued (the last one is in flight when in_flight)
    lf::GroupLaunch last{};         // iterating members of the launch in flight
    std::vector<lf_problem *> done; // finished runs not yet handed back
};

using namespace lf;

namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

size_t group_bytes(int32_t max_members) {
    return align256(sizeof(MemberDesc) * static_cast<size_t>(max_members)) +
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
    if (P->sp.grid_mx_amul != P->sp.grid_mx || P->sp.grid_amul != P->sp.grid) {
        set_error("unexpected product grid");
        return LF_EINVAL;
    }
    return LF_OK;
}

// the members of a launch, each with `count(member)` workgroups
template <class Count>
GroupLaunch launch_of(const lf_group *g, const std::vector<int32_t> &slots, Count &&count) {
    GroupLaunch gl{};
    int64_t blocks = 0;
    for (const int32_t s : slots) {
        gl.slot[gl.n] = s;
        gl.begin[gl.n] = static_cast<int32_t>(blocks);
        blocks += count(g->members[s]);
        ++gl.n;
    }
    gl.begin[gl.n] = static_cast<int32_t>(std::min<int64_t>(blocks, INT32_MAX));
    return gl;
}

// the member's step has ended (state h): its stats; the next launch copies T
// into the snapshot and starts the next step, or the run ends after that copy
void finish_step(GroupMember &m, const PcgState &h) {
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
    if (m.snap) m.snap_step = m.step;
    ++m.step;
    m.launched = 0;
    if (!h.nonfinite && m.step < m.n_steps) {
        m.start = true;
    } else {
        // the run ends: after the launch that copies its last snapshot, or at
        // once when there is none (no work of it is pending)
        m.final = true;
        m.final_launch = m.snap_step >= 0 ? -1 : 0;
    }
}

// the result of the launch that just finished
lf_status consume(lf_group *g) {
    for (int32_t i = 0; i < g->last.n; ++i) {
        GroupMember &m = g->members[g->last.slot[i]];
        const PcgState &h = g->h_states[g->last.slot[i]];
        m.launched += g->iters;
        if (h.done) {
            finish_step(m, h);
        } else if (m.launched > 4 * (static_cast<int64_t>(m.P->sp.max_iter) + 8) + 64 * m.P->sp.max_outer) {
            set_error("a member never reached the end of its solve after %lld inner iterations",
                      static_cast<long long>(m.launched));
            return LF_ESTATE;
        } else if (h.inner_done) {
            m.turn = true;          // its pass has ended
        }
    }
    // runs whose last snapshot copy has completed
    const int64_t completed = g->launches;
    for (auto &m : g->members) {
        if (!m.P || !m.final || m.final_launch < 0 || m.final_launch > completed) continue;
        m.P->group = nullptr;
        g->done.push_back(m.P);
        m = GroupMember{};
    }
    return LF_OK;
}

void add_copy(GroupCopy &gc, int64_t &blocks, int32_t cells, int32_t mode, const double *src, double *dst,
              const int32_t *perm) {
    const int32_t i = gc.n++;
    gc.cells[i] = cells;
    gc.mode[i] = mode;
    gc.src[i] = src;
    gc.dst[i] = dst;
    gc.perm[i] = perm;
    gc.begin[i] = static_cast<int32_t>(blocks);
    blocks += (cells + kBlock - 1) / kBlock;
    gc.begin[gc.n] = static_cast<int32_t>(blocks);
}

// the next launch: every member's pending copies, step starts and pass turns,
// then iters inner iterations of every iterating member and the gather of
// their states (nothing when no member has work)
lf_status launch_next(lf_group *g) {
    std::vector<int32_t> starts, turns, inner;
    GroupCopy out{}, in{};
    int64_t out_blocks = 0, in_blocks = 0;
    for (int32_t s = 0; s < g->max_members; ++s) {
        GroupMember &m = g->members[s];
        if (!m.P) continue;
        const lf_mesh *msh = m.P->mesh;
        if (m.snap_step >= 0) {
            add_copy(out, out_blocks, msh->N, msh->iperm ? 1 : 0, m.P->T,
                     m.snap + static_cast<int64_t>(m.snap_step) * msh->N, msh->iperm);
            m.snap_step = -1;
        }
        if (m.T0) {
            add_copy(in, in_blocks, msh->N, msh->iperm ? 2 : 0, m.T0, m.P->T, msh->iperm);
            m.T0 = nullptr;
        }
        if (m.start) starts.push_back(s);
        if (m.turn) turns.push_back(s);
        if (!m.final) inner.push_back(s);
    }
    const bool any_copy = out.n > 0 || in.n > 0;
    if (!any_copy && starts.empty() && turns.empty() && inner.empty()) return LF_OK;
    hipStream_t st = g->stream;
    if (out.n) hipLaunchKernelGGL(k_grp_copy, dim3(static_cast<unsigned>(out_blocks)), dim3(kBlock), 0, st, out);
    if (in.n) hipLaunchKernelGGL(k_grp_copy, dim3(static_cast<unsigned>(in_blocks)), dim3(kBlock), 0, st, in);
    const auto cells = [](const GroupMember &m) { return static_cast<int64_t>(m.P->sp.grid); };
    const auto inner_blocks = [](const GroupMember &m) { return static_cast<int64_t>(m.P->sp.grid_mx); };
    if (!starts.empty()) {
        const GroupLaunch gl = launch_of(g, starts, cells);
        launch_group_setup(g->d_tab, gl, st);
        launch_group_scale(g->d_tab, gl, st);
        launch_group_fin_start(g->d_tab, gl, st);
        launch_group_pass_start(g->d_tab, gl, st);
        for (const int32_t s : starts) {
            GroupMember &m = g->members[s];
            m.start = false;
            m.P->assembled = true;
            m.P->scaled32 = true;
        }
    }
    if (!turns.empty()) {
        const GroupLaunch gl = launch_of(g, turns, cells);
        launch_group_pass_end(g->d_tab, gl, st);
        launch_group_pass_start(g->d_tab, gl, st);
        for (const int32_t s : turns) g->members[s].turn = false;
    }
    GroupLaunch gi{};
    if (!inner.empty()) {
        gi = launch_of(g, inner, inner_blocks);
        for (int32_t k = 0; k < g->iters; ++k) launch_group_iteration(g->d_tab, gi, st);
        launch_group_gather(g->d_tab, gi, g->d_states, st);
        LF_HIP(hipMemcpyAsync(g->h_states, g->d_states, sizeof(PcgState) * static_cast<size_t>(g->max_members),
                              hipMemcpyDeviceToHost, st));
    }
    LF_HIP(hipGetLastError());
    LF_HIP(hipEventRecord(g->ev_block, st));
    ++g->launches;
    for (auto &m : g->members)
        if (m.P && m.final && m.final_launch < 0) m.final_launch = g->launches;
    g->in_flight = true;
    g->last = gi;
    return LF_OK;
}

void release(lf_group *g) {
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
    g->d_tab = reinterpret_cast<MemberDesc *>(base);
    g->d_states = reinterpret_cast<PcgState *>(base + align256(sizeof(MemberDesc) * max_members));
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&g->h_tab), sizeof(MemberDesc) * max_members,
                                           hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&g->h_states), sizeof(PcgState) * max_members,
                                           hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_block, hipEventDisableTiming);
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
        if (m.P) { set_error("members are still running"); return LF_ESTATE; }
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
        if (!g->members[s].P) slot = s;
    if (slot < 0) { set_error("the group is full (%d members)", g->max_members); return LF_EBUDGET; }
    // the problem's own earlier work (its T, its previous run) comes first
    hipEvent_t ev = P->ev[0];
    LF_HIP(hipEventRecord(ev, P->stream));
    LF_HIP(hipStreamWaitEvent(g->stream, ev, 0));
    // the descriptor, ordered on the group's stream before any launch reads it
    g->h_tab[slot] = member_desc(P);
    LF_HIP(hipMemcpyAsync(g->d_tab + slot, g->h_tab + slot, sizeof(MemberDesc), hipMemcpyHostToDevice, g->stream));
    GroupMember &m = g->members[slot];
    m = GroupMember{};
    m.P = P;
    m.n_steps = n_steps;
    m.snap = snapshots;
    m.stats = stats;
    m.T0 = T0;
    m.start = true;
    P->group = g;
    return LF_OK;
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
            LF_TRY(consume(g));
        } else if (q != hipErrorNotReady) {
            set_error("hipEventQuery failed: %s", hipGetErrorString(q));
            return LF_EDEVICE;
        }
    }
    if (!g->in_flight) LF_TRY(launch_next(g));
    const int32_t k = static_cast<int32_t>(std::min<size_t>(g->done.size(), static_cast<size_t>(max_finished)));
    for (int32_t i = 0; i < k; ++i) finished[i] = g->done[static_cast<size_t>(i)];
    g->done.erase(g->done.begin(), g->done.begin() + k);
    *n_finished = k;
    int32_t active = static_cast<int32_t>(g->done.size());
    for (const auto &m : g->members) active += m.P != nullptr;
    *n_active = active;
    return LF_OK;
}

}  // extern "C"
