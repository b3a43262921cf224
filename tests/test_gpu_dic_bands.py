"""DIC on the two-colour band layout (a red-black numbered box whose x-lines
hold an even number of cells): each face's coefficient stored once at its red
cell's direction slot, no column indices.

The rows visit their faces in the order of the sequential face loop, so the
matrix, the product and the DIC diagonal and sweeps are bitwise those of the
sliced row layout and of the oracle (the preconditioner's application is
compared in test_gpu_amg.py); time steps are compared with the oracle like the
other parity cases (1e-8, iterations within one) and with the row layout
(whose dot products sum the rows in another order).
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam, max_rel

pytestmark = pytest.mark.gpu

T_TOL = 1e-8


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _rb(nx, ny, nz, ratio=1.0):
    base = synth.box_mesh(nx, ny, nz, z_ratio=ratio)
    new_of_old, _ = synth.red_black_numbering(base)
    return synth.renumber(base, new_of_old), new_of_old


def _meshes():
    yield "rb_16x10x6_graded", _rb(16, 10, 6, 4.0)
    yield "rb_line_12", _rb(12, 1, 1)
    yield "rb_xy_10x6", _rb(10, 6, 1)
    yield "rb_xz_8x1x5", _rb(8, 1, 5, 3.0)
    yield "rb_4x4x4", _rb(4, 4, 4)
    yield "rb_34x20x9_graded", _rb(34, 20, 9, 10.0)       # several workgroups, ragged tail


MESHES = list(_meshes())
IDS = [n for n, _ in MESHES]
DT, dt = 2e-3, 5e-3


def _problem(L, mesh, layout=None, **kw):
    m = L.Mesh(mesh)
    opts = L.make_opts(precond=L.LF_PC_DIC, layout=L.LF_LAYOUT_AUTO if layout is None else layout, **kw)
    return m, L.Problem(m, synth.fixed_x_bcs(), DT, dt, opts)


@pytest.mark.parametrize("name,mm", MESHES, ids=IDS)
def test_rb_matrix_and_amul_bitwise(L, oracle, name, mm):
    import torch
    mesh, new_of_old = mm
    m, P = _problem(L, mesh)
    assert P.layout() == L.LF_LAYOUT_BANDS, name
    T0 = synth.initial_field(mesh.n_cells, 11, new_of_old=new_of_old)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        assert np.array_equal(g[k], o[k]), (name, k)
    x = np.random.default_rng(5).uniform(-1.0, 1.0, mesh.n_cells)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    P.amul(xd, yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), oracle.amul(mesh, o["diag_b"], o["upper"], x)), name
    P.close()
    m.close()


@pytest.mark.parametrize("name,mm", MESHES, ids=IDS)
def test_rb_steps_match_oracle_and_rows(L, oracle, name, mm):
    mesh, new_of_old = mm
    T0 = synth.initial_field(mesh.n_cells, 12, new_of_old=new_of_old)
    steps = 3
    _, so, snaps = oracle.run(mesh, synth.fixed_x_bcs(), DT, dt, steps, T0, pc=oracle.PC_DIC, keep_all=True)
    out = {}
    for layout in (L.LF_LAYOUT_AUTO, L.LF_LAYOUT_ROWS):
        m, P = _problem(L, mesh, layout)
        P.set_T(T0)
        Ts, st = [], []
        for s in range(steps):
            s1, _ = P.step(1)
            st += s1
            Ts.append(P.get_T())
        out[layout] = (Ts, st)
        P.close()
        m.close()
    Ts, st = out[L.LF_LAYOUT_AUTO]
    Tr, sr = out[L.LF_LAYOUT_ROWS]
    for s in range(steps):
        assert max_rel(Ts[s], snaps[s]) <= T_TOL, (name, s, max_rel(Ts[s], snaps[s]))
        assert abs(st[s]["n_iter"] - so[s]["n_iter"]) <= 1, (name, s)
        assert st[s]["converged"] == 1
        assert max_rel(Ts[s], Tr[s]) <= T_TOL, (name, s)
        assert abs(st[s]["n_iter"] - sr[s]["n_iter"]) <= 1, (name, s)


def test_rb_form_only_where_it_applies(L):
    """Odd x-lines (red and black counts differ per line), natural numbering
    and random numbering keep the row layout (or refuse DIC); asking for the
    band layout with DIC there is refused."""
    odd, _ = _rb(9, 6, 4)
    m = L.Mesh(odd)
    P = L.Problem(m, synth.fixed_x_bcs(), DT, dt, L.make_opts(precond=L.LF_PC_DIC))
    assert P.layout() == L.LF_LAYOUT_ROWS
    P.close()
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        L.Problem(m, synth.fixed_x_bcs(), DT, dt, L.make_opts(precond=L.LF_PC_DIC, layout=L.LF_LAYOUT_BANDS))
    m.close()
    even, _ = _rb(8, 6, 4)
    m = L.Mesh(even)
    # the diagonal preconditioner on a red-black mesh: rows (no band form of that kind)
    P = L.Problem(m, synth.fixed_x_bcs(), DT, dt)
    assert P.layout() == L.LF_LAYOUT_ROWS
    P.close()
    m.close()


# x-lines of a multiple of four cells (two red-black pairs per lane): boxes,
# a line and an xz box; 260 cells per line put a line's pairs on two waves
# (lanes at a wave's edge load their x-neighbours) and 8 lines on 17 waves
WALK_MESHES = [(n, mm) for n, mm in MESHES if n in ("rb_16x10x6_graded", "rb_4x4x4", "rb_line_12",
                                                   "rb_xz_8x1x5")]
WALK_MESHES.append(("rb_4x4x20", _rb(4, 4, 20)))
WALK_MESHES.append(("rb_260x4x2_graded", _rb(260, 4, 2, 3.0)))


@pytest.mark.parametrize("name,mm", WALK_MESHES, ids=[n for n, _ in WALK_MESHES])
def test_rb_walk_product_bitwise_and_steps(L, oracle, name, mm):
    """The assembly and the product with two red-black pairs per lane: matrix
    and product bitwise the oracle's; steps within 1e-8 of the oracle's
    sequential DIC and of the steps with one pair per thread, iterations
    within one."""
    import torch
    mesh, new_of_old = mm
    T0 = synth.initial_field(mesh.n_cells, 13, new_of_old=new_of_old)
    steps = 3
    _, so, snaps = oracle.run(mesh, synth.fixed_x_bcs(), DT, dt, steps, T0, pc=oracle.PC_DIC, keep_all=True)
    out = {}
    for walk in (L.LF_WALK_ON, L.LF_WALK_OFF):
        m, P = _problem(L, mesh, amul_walk=walk)
        assert P.layout() == L.LF_LAYOUT_BANDS
        assert P.amul_form() == (3 if walk == L.LF_WALK_ON else 0), name
        if walk == L.LF_WALK_ON:
            P.set_T(T0)
            P.assemble()
            o = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
            # the assembly in the same form: the matrix bitwise the oracle's
            g = P.matrix()
            for key in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
                assert np.array_equal(g[key], o[key]), (name, key)
            x = np.random.default_rng(7).uniform(-1.0, 1.0, mesh.n_cells)
            xd = torch.from_numpy(x).cuda()
            yd = torch.empty_like(xd)
            P.amul(xd, yd)
            torch.cuda.synchronize()
            assert np.array_equal(yd.cpu().numpy(), oracle.amul(mesh, o["diag_b"], o["upper"], x)), name
        P.set_T(T0)
        Ts, st = [], []
        for s in range(steps):
            s1, _ = P.step(1)
            st += s1
            Ts.append(P.get_T())
        out[walk] = (Ts, st)
        P.close()
        m.close()
    Tw, sw = out[L.LF_WALK_ON]
    Tp, sp = out[L.LF_WALK_OFF]
    for s in range(steps):
        assert max_rel(Tw[s], snaps[s]) <= T_TOL, (name, s, max_rel(Tw[s], snaps[s]))
        assert abs(sw[s]["n_iter"] - so[s]["n_iter"]) <= 1, (name, s)
        assert sw[s]["converged"] == 1
        assert max_rel(Tw[s], Tp[s]) <= T_TOL, (name, s)
        assert abs(sw[s]["n_iter"] - sp[s]["n_iter"]) <= 1, (name, s)
