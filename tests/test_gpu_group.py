"""Grouped stepping (lf_group_*): several precision-form problems whose inner
FP32 iterations share launches.  Each member's snapshots and stats must equal,
bit for bit, lf_step on the same problem alone (the members keep their own
workgroups, rows and fixed-order partial sums), whatever joins or leaves the
group meanwhile; the group refuses problems it cannot run and calls on running
members."""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _cases():
    """(name, mesh, bcs, DT, dt, seed, steps): band cubes of several sides, a
    graded box, a randomly numbered box (Morton order, row layout), one cell."""
    g = synth.box_mesh(14, 11, 9, z_ratio=3.0)
    rnd = synth.box_mesh(12, 10, 7)
    rnd = synth.renumber(rnd, synth.random_permutation(rnd.n_cells, 4))
    return [
        ("cube_16", synth.box_mesh(16, 16, 16), synth.fixed_x_bcs(), 3e-3, 1e-3, 11, 5),
        ("cube_33", synth.box_mesh(33, 33, 33), synth.fixed_x_bcs(), 1e-4, 1e-3, 12, 4),
        ("cube_24_fast", synth.box_mesh(24, 24, 24), synth.fixed_x_bcs(), 1e-2, 1e-3, 13, 6),
        ("graded_14x11x9", g, synth.fixed_x_bcs(), 2e-3, 2e-3, 14, 3),
        ("random_12x10x7", rnd, synth.fixed_x_bcs(), 1e-2, 1e-2, 15, 4),
        ("zero_gradient_9", synth.box_mesh(9, 9, 9), synth.all_zero_gradient(), 5e-3, 1e-3, 16, 3),
        ("one_cell", synth.box_mesh(1, 1, 1), synth.fixed_x_bcs(), 0.7, 0.3, 17, 2),
    ]


def _alone(L, mesh, bcs, DT, dt, T0, steps):
    """lf_step one step at a time: T (mesh order) and stats per step."""
    m = L.Mesh(mesh)
    P = L.Problem(m, bcs, DT, dt, L.make_opts(precision=L.LF_PREC_MIXED))
    P.set_T(T0)
    Ts, st = [], []
    for _ in range(steps):
        s, _ = P.step(1)
        st += s
        Ts.append(P.get_T())
    P.close()
    m.close()
    return Ts, st


def _run_group(L, cases, join_after=(), max_members=8, iters=0):
    """Run the cases as members of one group; case i joins once join_after[i]
    polls have passed (default 0).  Returns {name: (snapshots [steps][N], stats)}."""
    import torch
    streams = [torch.cuda.Stream() for _ in cases]
    G = L.Group(max_members, iters_per_block=iters, stream=torch.cuda.Stream())
    live, T0s = {}, {}
    for i, ((name, mesh, bcs, DT, dt, seed, steps), s) in enumerate(zip(cases, streams)):
        m = L.Mesh(mesh, stream=s)
        P = L.Problem(m, bcs, DT, dt, L.make_opts(precision=L.LF_PREC_MIXED), stream=s)
        assert P.amul_form() == 0
        T0 = synth.initial_field(mesh.n_cells, seed)
        if i % 2:
            # the run starts from a device T0 handed to lf_group_add, not the problem's T
            P.set_T(np.full(mesh.n_cells, 300.0))
            T0s[name] = torch.from_numpy(T0).cuda()
        else:
            P.set_T(T0)
        snaps = torch.full((steps, mesh.n_cells), float("nan"), dtype=torch.float64, device="cuda")
        live[name] = (m, P, snaps, steps)
    torch.cuda.synchronize()          # the snapshots' fill and the set-up are done
    out, pending, polls = {}, list(range(len(cases))), 0
    waits = list(join_after) + [0] * (len(cases) - len(join_after))
    by_handle = {}
    while pending or len(out) < len(cases):
        for i in list(pending):
            if polls >= waits[i]:
                name = cases[i][0]
                m, P, snaps, steps = live[name]
                G.add(P, steps, snaps, T0=T0s.get(name))
                by_handle[P.h.value] = name
                pending.remove(i)
        for P, stats in G.poll():
            name = by_handle[P.h.value]
            m, _, snaps, _ = live[name]
            torch.cuda.synchronize()
            out[name] = (snaps.cpu().numpy(), stats)
        polls += 1
        assert polls < 2_000_000, "group never finished"
    assert G.active == 0
    G.close()
    for name, (m, P, _, _) in live.items():
        P.close()
        m.close()
    return out


@pytest.mark.parametrize("iters", [0, 1, 7])
def test_group_equals_alone(L, iters):
    cases = _cases()
    ref = {c[0]: _alone(L, c[1], c[2], c[3], c[4], synth.initial_field(c[1].n_cells, c[5]), c[6]) for c in cases}
    # members join at different times (some while others are mid-run)
    got = _run_group(L, cases, join_after=(0, 0, 3, 7, 1, 20, 0), iters=iters)
    for name, steps_T in ref.items():
        Ts, st = steps_T
        snaps, gst = got[name]
        for s in range(len(Ts)):
            assert np.array_equal(snaps[s], Ts[s]), (name, s, max_rel(snaps[s], Ts[s]))
            for k in ("initial_residual", "final_residual", "n_iter", "converged", "nonfinite", "n_outer"):
                assert gst[s][k] == st[s][k], (name, s, k, gst[s][k], st[s][k])
            assert gst[s]["converged"] == 1


def test_group_alone_equals_mix_and_oracle(L, oracle):
    """One member alone in a group and in a full mix: the same bits, and each
    step within 1e-8 of the oracle's step from the same T."""
    cases = _cases()
    target = cases[1]
    alone = _run_group(L, [target])[target[0]]
    mix = _run_group(L, cases, join_after=(2, 0, 0, 0, 5, 0, 9))[target[0]]
    assert np.array_equal(alone[0], mix[0])
    name, mesh, bcs, DT, dt, seed, steps = target
    T_prev = synth.initial_field(mesh.n_cells, seed)
    for s in range(steps):
        ref, _, _ = oracle.run(mesh, bcs, DT, dt, 1, T_prev)
        assert max_rel(mix[0][s], ref) <= 1e-8, (s, max_rel(mix[0][s], ref))
        T_prev = mix[0][s]


def test_group_refusals(L):
    import torch
    mesh = synth.box_mesh(10, 9, 8)
    m = L.Mesh(mesh)
    G = L.Group(2)
    T0 = synth.initial_field(mesh.n_cells, 3)
    # not the precision form, or not the product the group runs
    for opts in (dict(), dict(precision=L.LF_PREC_MIXED, amul_walk=L.LF_WALK_ON)):
        P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(**opts))
        P.set_T(T0)
        with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
            G.add(P, 2)
        P.close()
    Ps = [L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(precision=L.LF_PREC_MIXED)) for _ in range(3)]
    for P in Ps:
        P.set_T(T0)
    G.add(Ps[0], 3)
    with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
        G.add(Ps[0], 3)                       # runs already
    with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
        Ps[0].set_T(T0)                       # a running member is not set
    with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
        Ps[0].step(1)
    with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
        L.lf_problem_destroy(Ps[0].h)
    G.add(Ps[1], 2)
    with pytest.raises(L.LapfoamError, match="LF_EBUDGET"):
        G.add(Ps[2], 2)                       # full
    with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
        L.lf_group_destroy(G.h)               # members running
    finished = []
    for _ in range(1_000_000):
        finished += G.poll()
        if len(finished) == 2:
            break
    assert len(finished) == 2 and G.active == 0
    # finished members are usable again
    Ps[0].set_T(T0)
    Ps[0].step(1)
    torch.cuda.synchronize()
    G.close()
    for P in Ps:
        P.close()
    m.close()
