"""Batched persistent form: many independent problems in one launch.

Each problem's step agrees with the FP64 oracle's solve of the same system to
1e-8 max relative error, its FP64 true residual is below the tolerance, and its
result is bitwise the same alone, in a mix, and with any number of workgroups
(the reductions run in a fixed order inside one workgroup).
"""
import numpy as np
import pytest

import synth
from synth import FIXED_VALUE, ZERO_GRADIENT
from tests.gpu_common import lapfoam, max_rel

pytestmark = pytest.mark.gpu

T_TOL = 1e-8


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _requests(k, seed=0):
    """k small heat problems with varied sides, DT, boundary conditions."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(rng.integers(5, 22))
        nz = int(rng.integers(3, 14))
        mesh = synth.box_mesh(n, max(1, n - 3), nz, z_ratio=float(rng.choice([1.0, 4.0])))
        if i % 3 == 2:
            mesh = synth.renumber(mesh, synth.random_permutation(mesh.n_cells, i))
        DT = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        bcs = synth.fixed_x_bcs() if i % 4 else [(FIXED_VALUE, 300.0), (ZERO_GRADIENT, 0.0),
                                                 (FIXED_VALUE, 500.0), (ZERO_GRADIENT, 0.0),
                                                 (ZERO_GRADIENT, 0.0), (ZERO_GRADIENT, 0.0)]
        T0 = synth.initial_field(mesh.n_cells, 1000 + i)
        out.append((mesh, bcs, DT, 1e-3, T0))
    return out


def _run(L, reqs, steps, bs=512, n_wg=0, order=None, layout=None):
    import torch
    order = list(range(len(reqs))) if order is None else order
    meshes, probs, snaps = [], [], []
    for i in order:
        mesh, bcs, DT, dt, T0 = reqs[i]
        m = L.Mesh(mesh)
        lay = L.LF_LAYOUT_ROWS if layout is None else layout
        if lay == L.LF_LAYOUT_AUTO and m.n_bands not in (0, 3):
            lay = L.LF_LAYOUT_ROWS                     # the batched band layout is for 3-band meshes
        P = L.Problem(m, bcs, DT, dt, L.make_opts(precision=L.LF_PREC_MIXED, layout=lay))
        P.set_T(T0)
        meshes.append(m)
        probs.append(P)
        snaps.append(torch.empty(steps * mesh.n_cells, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    b = L.Batch(len(probs), steps)
    b.launch(probs, steps, block_threads=bs, n_workgroups=n_wg, snapshots=snaps)
    b.wait()
    stats, ms = b.stats()
    res = {}
    for k, i in enumerate(order):
        res[i] = (snaps[k].cpu().numpy().reshape(steps, -1), stats[k], probs[k].get_T())
    for P in probs:
        P.close()
    for m in meshes:
        m.close()
    b.close()
    return res


@pytest.mark.parametrize("layout", ["rows", "auto"])
def test_batch_matches_oracle(L, oracle, layout):
    reqs = _requests(12, seed=1)
    steps = 3
    res = _run(L, reqs, steps, layout=L.LF_LAYOUT_ROWS if layout == "rows" else L.LF_LAYOUT_AUTO)
    for i, (mesh, bcs, DT, dt, T0) in enumerate(reqs):
        snaps, stats, T_final = res[i]
        assert np.array_equal(snaps[-1], T_final)
        T_prev = T0
        for s in range(steps):
            ref, so, _ = oracle.run(mesh, bcs, DT, dt, 1, T_prev)
            assert max_rel(snaps[s], ref) <= T_TOL, (i, s, max_rel(snaps[s], ref))
            assert stats[s]["converged"] == 1 and stats[s]["final_residual"] < 1e-10
            assert abs(stats[s]["initial_residual"] - so[0]["initial_residual"]) <= \
                1e-9 * so[0]["initial_residual"]
            m = oracle.assemble(mesh, bcs, DT, dt, T_prev)
            r = m["source_b"] - oracle.amul(mesh, m["diag_b"], m["upper"], snaps[s])
            A1 = oracle.sum_a(mesh, m["diag_b"], m["upper"])
            pA = A1 * T_prev.mean()
            Ax0 = oracle.amul(mesh, m["diag_b"], m["upper"], T_prev)
            nf = np.sum(np.abs(Ax0 - pA) + np.abs(m["source_b"] - pA)) + 1e-20
            assert np.sum(np.abs(r)) / nf < 1e-9
            T_prev = snaps[s]


@pytest.mark.parametrize("bs,layout", [(256, "rows"), (1024, "rows"), (512, "auto")])
def test_alone_equals_in_mix(L, bs, layout):
    lay = L.LF_LAYOUT_ROWS if layout == "rows" else L.LF_LAYOUT_AUTO
    reqs = _requests(10, seed=2)
    steps = 2
    mix = _run(L, reqs, steps, bs=bs, layout=lay)
    shuffled = _run(L, reqs, steps, bs=bs, order=[9, 3, 0, 7, 1, 8, 2, 6, 4, 5], n_wg=3, layout=lay)
    for i in (0, 4, 9):
        alone = _run(L, [reqs[i]], steps, bs=bs, layout=lay)[0]
        assert np.array_equal(alone[0], mix[i][0])
        assert np.array_equal(alone[0], shuffled[i][0])
        assert alone[1] == mix[i][1]


def test_batch_edge_cases(L, oracle):
    # zero diffusivity (no pass), one cell, a line, all zeroGradient
    reqs = [
        (synth.box_mesh(6, 5, 4), synth.fixed_x_bcs(), 0.0, 1e-3, synth.initial_field(120, 1)),
        (synth.box_mesh(1, 1, 1), synth.fixed_x_bcs(), 0.3, 0.2, np.array([400.0])),
        (synth.box_mesh(40, 1, 1), synth.fixed_x_bcs(), 0.1, 0.01, synth.initial_field(40, 2)),
        (synth.box_mesh(7, 6, 5, z_ratio=3.0), synth.all_zero_gradient(), 0.01, 0.01,
         synth.initial_field(210, 3)),
    ]
    res = _run(L, reqs, 2, bs=256)
    assert res[0][1][0]["n_iter"] == 0 and res[0][1][0]["n_outer"] == 0
    for i, (mesh, bcs, DT, dt, T0) in enumerate(reqs):
        ref, _, _ = oracle.run(mesh, bcs, DT, dt, 1, T0)
        assert max_rel(res[i][0][0], ref) <= T_TOL, i


def test_batch_refuses_bad_input(L):
    mesh = synth.box_mesh(4, 4, 4)
    m = L.Mesh(mesh)
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3)          # FP64: not accepted
    b = L.Batch(2, 2)
    with pytest.raises(L.LapfoamError):
        b.launch([P], 1)
    Pm = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3,
                   L.make_opts(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_ROWS))
    with pytest.raises(L.LapfoamError):
        b.launch([Pm, Pm, Pm], 1)                                # more than max_tasks
    with pytest.raises(L.LapfoamError):
        b.launch([Pm], 3)                                        # more than max_steps
    with pytest.raises(L.LapfoamError):
        b.launch([Pm], 1, block_threads=128)
    flat = L.Mesh(synth.box_mesh(6, 5, 1))                     # 2 bands: not batched in bands
    assert flat.n_bands == 2
    Pb = L.Problem(flat, synth.fixed_x_bcs(), 1e-3, 1e-3,
                   L.make_opts(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_BANDS))
    with pytest.raises(L.LapfoamError):
        b.launch([Pb], 1)
    Pb.close()
    flat.close()
    b.close()
    P.close()
    Pm.close()
    m.close()


def test_batch_at_served_sizes(L, oracle):
    """The cube sides the serving stream puts on the batched kernel (24..31,
    up to 29,791 cells; band layout, the tuned workgroup size of the bucket):
    each step against the oracle's step from the same T, and each problem
    bitwise the same alone and in the mix."""
    from paper_2507_18268_amd import autotune
    rng = np.random.default_rng(12)
    reqs = []
    for i, n in enumerate((24, 26, 29, 31)):
        DT = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        reqs.append((synth.box_mesh(n, n, n), synth.fixed_x_bcs(), DT, 1e-3,
                     synth.initial_field(n ** 3, 7000 + i)))
    bs = autotune.block_threads_for(24)
    assert all(autotune.block_threads_for(r[0].shape[0]) == bs for r in reqs)
    steps = 3
    mix = _run(L, reqs, steps, bs=bs, layout=L.LF_LAYOUT_AUTO)
    for i, (mesh, bcs, DT, dt, T0) in enumerate(reqs):
        snaps, stats, _ = mix[i]
        T_prev = T0
        for s in range(steps):
            ref, _, _ = oracle.run(mesh, bcs, DT, dt, 1, T_prev)
            assert max_rel(snaps[s], ref) <= T_TOL, (mesh.shape, s, max_rel(snaps[s], ref))
            assert stats[s]["converged"] == 1
            T_prev = snaps[s]
    for i in (0, 3):
        alone = _run(L, [reqs[i]], steps, bs=bs, layout=L.LF_LAYOUT_AUTO)[0]
        assert np.array_equal(alone[0], mix[i][0])
