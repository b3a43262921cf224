"""FP64 solves with the diagonal preconditioner in product form 4: CG on the
Jacobi-scaled system S A S (S = diag(1/sqrt(diagB)), unit diagonal) over the
block walk, taken by boxes whose iteration reductions are not folded into the
update and direction (more than 512 partials per slot: above about 1 M cells).

In exact arithmetic the scaled iteration has the iterates of the diagonally
preconditioned CG, so its steps are held to the bar of the other parity cases:
T within 1e-8 (max relative) of the oracle's, iterations within one, the
initial residual (of A, taken before scaling) within 1e-10; and likewise
against the unscaled one-row-per-thread path of the same problem.  The matrix
and the product hook (A, not S A S) stay bitwise the oracle's after steps.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam, max_rel

pytestmark = pytest.mark.gpu

T_TOL = 1e-8
DT, dt = 5e-3, 2e-3


@pytest.fixture(scope="module")
def L():
    return lapfoam()


# 128x96x96 graded: tiles whole; 130x97x91: x-lines wider than a wavefront's
# rows, ragged tiles in y and z; 110x100x100 at the paper's DT and dt
BOXES = [((128, 96, 96, 10.0), DT, dt, 3), ((130, 97, 91, 4.0), DT, dt, 3),
         ((110, 100, 100, 1.0), 1e-4, 0.2, 2)]
IDS = ["graded_128x96x96", "ragged_130x97x91", "paper_dt_110x100x100"]


def _steps(L, mesh, DTs, dts, T0, steps, **kw):
    m = L.Mesh(mesh)
    P = L.Problem(m, synth.fixed_x_bcs(), DTs, dts, L.make_opts(**kw))
    form = P.amul_form()
    P.set_T(T0)
    Ts, st = [], []
    for _ in range(steps):
        s1, _ = P.step(1)
        st += s1
        Ts.append(P.get_T())
    return m, P, form, Ts, st


@pytest.mark.parametrize("box,DTs,dts,steps", BOXES, ids=IDS)
def test_scaled_steps_match_oracle_and_unscaled(L, oracle, box, DTs, dts, steps):
    nx, ny, nz, ratio = box
    mesh = synth.box_mesh(nx, ny, nz, z_ratio=ratio)
    T0 = synth.initial_field(mesh.n_cells, 31)
    _, so, snaps = oracle.run(mesh, synth.fixed_x_bcs(), DTs, dts, steps, T0, keep_all=True)
    m, P, form, Ts, st = _steps(L, mesh, DTs, dts, T0, steps, amul_walk=L.LF_WALK_ON)
    assert form == 4, form
    P.close()
    m.close()
    m, P, form0, Tu, su = _steps(L, mesh, DTs, dts, T0, steps, amul_walk=L.LF_WALK_OFF)
    assert form0 == 0
    P.close()
    m.close()
    for s in range(steps):
        assert max_rel(Ts[s], snaps[s]) <= T_TOL, (box, s, max_rel(Ts[s], snaps[s]))
        assert abs(st[s]["n_iter"] - so[s]["n_iter"]) <= 1, (box, s, st[s], so[s])
        assert st[s]["converged"] == 1 and st[s]["final_residual"] < 1e-9
        assert abs(st[s]["initial_residual"] - so[s]["initial_residual"]) <= 1e-10 * so[s]["initial_residual"]
        assert max_rel(Ts[s], Tu[s]) <= T_TOL, (box, s)
        assert abs(st[s]["n_iter"] - su[s]["n_iter"]) <= 1, (box, s)


def test_scaled_leaves_matrix_and_product_hook_of_A(L, oracle):
    """After scaled steps the stored matrix is A's, and the hook multiplies by
    A bitwise (the scaled coefficients live in their own array)."""
    import torch
    mesh = synth.box_mesh(128, 96, 96, z_ratio=10.0)
    T0 = synth.initial_field(mesh.n_cells, 32)
    m, P, form, Ts, _ = _steps(L, mesh, DT, dt, T0, 2, amul_walk=L.LF_WALK_ON)
    assert form == 4
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, Ts[-1])
    for k in ("diag", "upper", "source", "diag_b", "source_b"):
        assert np.array_equal(g[k], o[k]), k
    x = np.random.default_rng(9).uniform(-1.0, 1.0, mesh.n_cells)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    P.amul(xd, yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), oracle.amul(mesh, o["diag_b"], o["upper"], x))
    P.close()
    m.close()


def test_scaled_graph_blocks_bitwise_and_edges(L, oracle):
    """Graph blocks and single launches give bitwise the same steps; a solve
    that starts converged leaves T bitwise untouched (no iteration: the commit
    does not rescale); a solve stopped by max_iter matches the oracle's."""
    mesh = synth.box_mesh(130, 97, 91, z_ratio=4.0)
    T0 = synth.initial_field(mesh.n_cells, 33)
    runs = []
    for kw in (dict(), dict(use_graph=0), dict(use_graph=0, iters_per_check=3)):
        m, P, form, Ts, st = _steps(L, mesh, DT, dt, T0, 2, amul_walk=L.LF_WALK_ON, **kw)
        assert form == 4
        runs.append((Ts, st))
        P.close()
        m.close()
    for Ts, st in runs[1:]:
        for s in range(2):
            assert np.array_equal(Ts[s], runs[0][0][s]), s
            assert st[s]["n_iter"] == runs[0][1][s]["n_iter"]
    m, P, form, Ts, st = _steps(L, mesh, DT, dt, T0, 1, amul_walk=L.LF_WALK_ON, tol=1e30)
    assert form == 4 and st[0]["n_iter"] == 0
    assert np.array_equal(Ts[0], T0)
    P.close()
    m.close()
    m, P, form, Ts, st = _steps(L, mesh, DT, dt, T0, 1, amul_walk=L.LF_WALK_ON, max_iter=2)
    assert form == 4 and st[0]["n_iter"] == 2 and st[0]["converged"] == 0
    To, so, _ = oracle.run(mesh, synth.fixed_x_bcs(), DT, dt, 1, T0, max_iter=2)
    assert so[0]["n_iter"] == 2
    assert max_rel(Ts[0], To) <= T_TOL, max_rel(Ts[0], To)
    P.close()
    m.close()


def test_scaled_corrected_steps_on_skewed_box(L, oracle):
    """The non-orthogonal correction with one extra corrector pass per step:
    each pass's solve in the scaled form, against the oracle's passes."""
    mesh = synth.affine(synth.box_mesh(128, 96, 96, z_ratio=10.0), synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    P = L.Problem(m, synth.fixed_x_bcs(), DT, dt, L.make_opts(amul_walk=L.LF_WALK_ON, n_nonorth_corr=1))
    assert P.amul_form() == 4
    T0 = synth.initial_field(mesh.n_cells, 34)
    P.set_T(T0)
    steps = 2
    _, so, snaps = oracle.run_nonorth(mesh, synth.fixed_x_bcs(), DT, dt, steps, T0, n_corr=1)
    for s in range(steps):
        st, _ = P.step(1)
        T = P.get_T()
        assert max_rel(T, snaps[s]) <= T_TOL, (s, max_rel(T, snaps[s]))
        assert abs(st[0]["n_iter"] - so[s]["n_iter"]) <= 3, (s, st[0], so[s])
    P.close()
    m.close()


def test_scaled_by_default_on_a_4m_box(L, oracle):
    """A 170x160x160 box (4.35 M cells, 2125 block-walk workgroups) takes the
    block walk and the scaled solve with the default options (the row walk
    alone would not fill the GPU): one step against the oracle's."""
    mesh = synth.box_mesh(170, 160, 160, z_ratio=10.0)
    T0 = synth.initial_field(mesh.n_cells, 35)
    m, P, form, Ts, st = _steps(L, mesh, DT, dt, T0, 1)
    assert form == 4, form
    P.close()
    m.close()
    To, so, _ = oracle.run(mesh, synth.fixed_x_bcs(), DT, dt, 1, T0)
    assert max_rel(Ts[0], To) <= T_TOL, max_rel(Ts[0], To)
    assert abs(st[0]["n_iter"] - so[0]["n_iter"]) <= 1, (st[0], so[0])
    assert st[0]["converged"] == 1


def test_scaled_step_begin_poll_equals_step(L):
    """lf_step_begin / lf_step_poll on a problem in the scaled form: bitwise the
    snapshots and stats of stepping one step at a time."""
    import torch
    mesh = synth.box_mesh(130, 97, 91, z_ratio=4.0)
    N = mesh.n_cells
    T0 = synth.initial_field(N, 36)
    steps = 3
    m, A, form, ref, sref = _steps(L, mesh, DT, dt, T0, steps, amul_walk=L.LF_WALK_ON)
    assert form == 4
    B = L.Problem(m, synth.fixed_x_bcs(), DT, dt, L.make_opts(amul_walk=L.LF_WALK_ON))
    B.set_T(T0)
    snap = torch.empty(steps * N, dtype=torch.float64, device="cuda")
    B.step_begin(steps, snap)
    while True:
        done, finished, stats, status = B.step_poll()
        if finished:
            break
    assert status == L.LF_OK and done == steps
    got = snap.view(steps, N).cpu().numpy()
    for s in range(steps):
        assert np.array_equal(got[s], ref[s]), s
        assert stats[s]["n_iter"] == sref[s]["n_iter"]
        assert stats[s]["final_residual"] == sref[s]["final_residual"]
    A.close()
    B.close()
    m.close()
