"""The multigrid preconditioner (LF_PC_AMG) and the preconditioner hook on the
GPU against the oracle.

The cycle sums every level's matrix, residuals and corrections in the order of
the sequential definition, so one application w = M r (lf_precondition) is
compared bit for bit with the oracle's cycle on the same assembled matrix and
the box's 2x2x2 aggregation; the DIC and diagonal preconditioners likewise.
Time steps are compared like the other parity cases (1e-8, iterations within
one).
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


# sides even and odd; the levels of a box with even x-lines take the block
# walk (and the restriction too when all its sides are even): 64^3 on every
# level, 130x4x4 with x-lines wider than a wavefront's rows
BOXES = [(12, 10, 8, 4.0), (24, 20, 18, 10.0), (40, 33, 17, 3.0), (2, 2, 2, 1.0), (64, 64, 64, 10.0),
         (130, 4, 4, 2.0)]
IDS = ["x".join(str(v) for v in b[:3]) for b in BOXES]


def _run_hook(L, mesh, T0, pc, layout=None, **kw):
    import torch
    m = L.Mesh(mesh)
    opts = L.make_opts(precond=pc, **kw) if layout is None else L.make_opts(precond=pc, layout=layout, **kw)
    P = L.Problem(m, synth.fixed_x_bcs(), DT, dt, opts)
    P.set_T(T0)
    P.assemble()
    r = np.random.default_rng(7).uniform(-1.0, 1.0, mesh.n_cells)
    rd = torch.from_numpy(r).cuda()
    wd = torch.empty_like(rd)
    P.precondition(rd, wd)
    torch.cuda.synchronize()
    out = wd.cpu().numpy()
    P.close()
    m.close()
    return r, out


@pytest.mark.parametrize("walk", [0, 1, 2], ids=["auto", "walk", "nowalk"])
@pytest.mark.parametrize("box", BOXES, ids=IDS)
def test_amg_cycle_bitwise(L, oracle, box, walk):
    """One application bitwise the oracle's cycle with the sweeps, the
    restriction and the prolongation by the block walk on every level with
    even x-lines (LF_WALK_ON), on none (LF_WALK_OFF), and as chosen by size."""
    nx, ny, nz, ratio = box
    mesh = synth.box_mesh(nx, ny, nz, z_ratio=ratio)
    T0 = synth.initial_field(mesh.n_cells, 17)
    r, w = _run_hook(L, mesh, T0, L.LF_PC_AMG, amul_walk=walk)
    A = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    lc, ag = synth.box_aggregation((nx, ny, nz))
    want = oracle.amg_apply(mesh, A["diag_b"], A["upper"], r, lc, ag)
    assert np.array_equal(w, want), (box, len(lc), float(np.max(np.abs(w - want))))


@pytest.mark.parametrize("name,mesh,layout", [
    ("rows_redblack_9x6x4", synth.renumber(synth.box_mesh(9, 6, 4), synth.red_black_numbering(synth.box_mesh(9, 6, 4))[0]), None),
    ("bands_redblack_16x10x6", synth.renumber(synth.box_mesh(16, 10, 6, z_ratio=3.0),
                                              synth.red_black_numbering(synth.box_mesh(16, 10, 6))[0]), None),
    ("rows_redblack_16x10x6", synth.renumber(synth.box_mesh(16, 10, 6, z_ratio=3.0),
                                             synth.red_black_numbering(synth.box_mesh(16, 10, 6))[0]), 1),
    # the two-colour band layout with two red-black pairs per lane (DIC diagonal and sweeps)
    ("pairs_redblack_16x10x6", synth.renumber(synth.box_mesh(16, 10, 6, z_ratio=3.0),
                                              synth.red_black_numbering(synth.box_mesh(16, 10, 6))[0]), "pairs"),
    ("pairs_redblack_260x4x3", synth.renumber(synth.box_mesh(260, 4, 3, z_ratio=2.0),
                                              synth.red_black_numbering(synth.box_mesh(260, 4, 3))[0]), "pairs"),
])
def test_dic_application_bitwise(L, oracle, name, mesh, layout):
    T0 = synth.initial_field(mesh.n_cells, 18)
    if layout == "pairs":
        r, w = _run_hook(L, mesh, T0, L.LF_PC_DIC, amul_walk=L.LF_WALK_ON)
    else:
        r, w = _run_hook(L, mesh, T0, L.LF_PC_DIC, layout)
    A = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    rd = oracle.dic_rd(mesh, A["diag_b"], A["upper"])
    want = oracle.precondition(mesh, oracle.PC_DIC, A["upper"], rd, r)
    assert np.array_equal(w, want), name


def test_diagonal_application_bitwise(L, oracle):
    base = synth.box_mesh(11, 9, 7, z_ratio=2.0)
    for mesh in (base, synth.renumber(base, synth.random_permutation(base.n_cells, 4))):
        T0 = synth.initial_field(mesh.n_cells, 19)
        r, w = _run_hook(L, mesh, T0, L.LF_PC_DIAGONAL)
        A = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
        want = oracle.precondition(mesh, oracle.PC_DIAGONAL, A["upper"], 1.0 / A["diag_b"], r)
        assert np.array_equal(w, want)


@pytest.mark.parametrize("box,steps,DTs,dts", [((24, 20, 18, 10.0), 4, 5e-3, 2e-3),
                                               ((33, 30, 28, 1.0), 3, 1e-2, 0.2),
                                               ((12, 10, 8, 4.0), 3, 5e-3, 2e-3)],
                         ids=["graded_24x20x18", "paper_dt_33x30x28", "two_levels_12x10x8"])
@pytest.mark.parametrize("walk", [0, 1], ids=["auto", "walk"])
def test_amg_steps_match_oracle(L, oracle, box, steps, DTs, dts, walk):
    nx, ny, nz, ratio = box
    mesh = synth.box_mesh(nx, ny, nz, z_ratio=ratio)
    T0 = synth.initial_field(mesh.n_cells, 20)
    lc, ag = synth.box_aggregation((nx, ny, nz))
    _, so, snaps = oracle.run_amg(mesh, synth.fixed_x_bcs(), DTs, dts, steps, T0, lc, ag, keep_all=True)
    _, sd, _ = oracle.run(mesh, synth.fixed_x_bcs(), DTs, dts, steps, T0)
    m = L.Mesh(mesh)
    P = L.Problem(m, synth.fixed_x_bcs(), DTs, dts, L.make_opts(precond=L.LF_PC_AMG, amul_walk=walk))
    P.set_T(T0)
    for s in range(steps):
        st, _ = P.step(1)
        T = P.get_T()
        assert max_rel(T, snaps[s]) <= T_TOL, (s, max_rel(T, snaps[s]))
        assert abs(st[0]["n_iter"] - so[s]["n_iter"]) <= 1, (s, st[0], so[s])
        assert st[0]["converged"] == 1 and st[0]["final_residual"] < 1e-9
        assert so[s]["n_iter"] < sd[s]["n_iter"]          # the cycle beats the diagonal preconditioner
    P.close()
    m.close()


def test_amg_refused_where_it_does_not_apply(L):
    base = synth.box_mesh(8, 6, 5)
    cases = [(synth.renumber(base, synth.random_permutation(base.n_cells, 2)), {}),   # no box form
             (base, dict(layout=L.LF_LAYOUT_ROWS)),
             (base, dict(precision=L.LF_PREC_MIXED)),
             (synth.box_mesh(8, 6, 1), {})]                                         # a plane: 2 bands
    for mesh, kw in cases:
        m = L.Mesh(mesh)
        with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
            L.Problem(m, synth.fixed_x_bcs(), DT, dt, L.make_opts(precond=L.LF_PC_AMG, **kw))
        m.close()
