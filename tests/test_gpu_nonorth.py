"""Time steps on skewed meshes: the Laplacian's explicit non-orthogonal
correction (gradient of T, interpolated to the faces, dotted with the faces'
correction vectors, divergence subtracted from TEqn's source) on the GPU
against the oracle's corrected step.

The assembled matrix and source are compared bit for bit (the correction is
summed in the face loop's order); time steps within 1e-8 (max relative) and
iteration counts within one, as for orthogonal meshes.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam, max_rel
from tests.helpers import tiny_face_cells

pytestmark = pytest.mark.gpu

BCS = synth.fixed_x_bcs()


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _meshes():
    skew = lambda m: synth.affine(m, synth.SKEW)
    g = synth.box_mesh(9, 8, 7, z_ratio=4.0)
    yield "skew_graded_9x8x7", skew(g), "diagonal"
    yield "skew_random_9x8x7", skew(synth.renumber(g, synth.random_permutation(g.n_cells, 3))), "diagonal"
    rb = synth.box_mesh(6, 5, 4, z_ratio=2.0)
    yield "skew_redblack_6x5x4_dic", skew(synth.renumber(rb, synth.red_black_numbering(rb)[0])), "dic"
    yield "skew_line_9", skew(synth.box_mesh(9, 1, 1)), "diagonal"
    yield "skew_one_cell", skew(synth.box_mesh(1, 1, 1)), "diagonal"
    big = synth.box_mesh(20, 17, 13, z_ratio=10.0)
    yield "skew_random_20x17x13", skew(synth.renumber(big, synth.random_permutation(big.n_cells, 8))), "diagonal"
    # x and y faces past the limiter's angle: delta_f = 1/(0.05|d|) (band form, rows, red-black)
    steep = lambda m: synth.affine(m, synth.STEEP)
    yield "steep_graded_9x8x7", steep(g), "diagonal"
    yield "steep_random_9x8x7", steep(synth.renumber(g, synth.random_permutation(g.n_cells, 5))), "diagonal"
    yield "steep_redblack_6x5x4_dic", steep(synth.renumber(rb, synth.red_black_numbering(rb)[0])), "dic"


MESHES = list(_meshes())
IDS = [n for n, _, _ in MESHES]
DT, dt = 2e-3, 5e-3


def _problem(L, mesh, pc, **kw):
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    pcc = L.LF_PC_DIC if pc == "dic" else L.LF_PC_DIAGONAL
    P = L.Problem(m, BCS, DT, dt, L.make_opts(precond=pcc, **kw))
    return m, P


@pytest.mark.parametrize("name,mesh,pc", MESHES, ids=IDS)
def test_nonorth_matrix_bitwise(L, oracle, name, mesh, pc):
    m, P = _problem(L, mesh, pc)
    T0 = synth.initial_field(mesh.n_cells, 5)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    lap_src = oracle.step_source(mesh, BCS, DT, T0)
    o = oracle.assemble(mesh, BCS, DT, dt, T0, lap_src=lap_src)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        assert np.array_equal(g[k], o[k]), (name, k, float(np.max(np.abs(g[k] - o[k]))))
    if mesh.n_faces:
        assert np.max(np.abs(lap_src)) > 0.0
    P.close()
    m.close()


def test_nonorth_matrix_tiny_face_bitwise(L, oracle):
    """Two cells whose face takes the interpolation weight's fallback (1/2) and
    the limiter: the correction (weights, k_f, delta_f) bit for bit."""
    mesh = tiny_face_cells()
    m, P = _problem(L, mesh, "diagonal")
    T0 = np.array([300.0, 500.0])
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    lap_src = oracle.step_source(mesh, BCS, DT, T0)
    o = oracle.assemble(mesh, BCS, DT, dt, T0, lap_src=lap_src)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        assert np.array_equal(g[k], o[k]), (k, g[k], o[k])
    assert np.max(np.abs(lap_src)) > 0.0
    P.close()
    m.close()


@pytest.mark.parametrize("name,mesh,pc", MESHES, ids=IDS)
def test_nonorth_steps_match_oracle(L, oracle, name, mesh, pc):
    m, P = _problem(L, mesh, pc)
    T0 = synth.initial_field(mesh.n_cells, 6)
    P.set_T(T0)
    steps = 4
    _, ostats, osnaps = oracle.run_nonorth(mesh, BCS, DT, dt, steps, T0,
                                           pc=oracle.PC_DIC if pc == "dic" else oracle.PC_DIAGONAL)
    for s in range(steps):
        st, _ = P.step(1)
        T = P.get_T()
        assert max_rel(T, osnaps[s]) <= 1e-8, (name, s, max_rel(T, osnaps[s]))
        assert abs(st[0]["n_iter"] - ostats[s]["n_iter"]) <= 1, (name, s)
    P.close()
    m.close()


def test_nonorth_mixed_precision_per_step(L, oracle):
    """The precision form on a skewed box: each step against the oracle's
    corrected step from the same T."""
    mesh = synth.affine(synth.box_mesh(14, 12, 10, z_ratio=5.0), synth.SKEW)
    m, P = _problem(L, mesh, "diagonal", precision=L.LF_PREC_MIXED)
    T = synth.initial_field(mesh.n_cells, 7)
    P.set_T(T)
    for s in range(3):
        P.step(1)
        Tg = P.get_T()
        To, _, _ = oracle.run_nonorth(mesh, BCS, DT, dt, 1, T)
        assert max_rel(Tg, To) <= 1e-8, (s, max_rel(Tg, To))
        T = Tg
    P.close()
    m.close()


def test_batch_refuses_nonorth_problem(L):
    mesh = synth.affine(synth.box_mesh(4, 4, 4), synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    P = L.Problem(m, BCS, DT, dt, L.make_opts(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_ROWS))
    B = L.Batch(4, 2)
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        B.launch([P], 1)
    B.close()
    P.close()
    m.close()


def test_nonorth_full_size_skewed_256(L, oracle):
    """The 256^3 box graded in z, skewed: the corrected matrix and source bit
    for bit, and one step within 1e-8 of the oracle's."""
    p = synth.build_config("graded_256")
    mesh = synth.affine(p.mesh, synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    opts = L.make_opts(tol=synth.TOL, rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER)
    P = L.Problem(m, p.bcs, p.DT, p.dt, opts)
    P.set_T(p.T0)
    P.assemble()
    g = P.matrix()
    lap_src = oracle.step_source(mesh, p.bcs, p.DT, p.T0)
    o = oracle.assemble(mesh, p.bcs, p.DT, p.dt, p.T0, lap_src=lap_src)
    for k in ("diag", "source", "diag_b", "source_b"):
        assert np.array_equal(g[k], o[k]), k
    del g
    st, _ = P.step(1)
    T = P.get_T()
    P.close()
    m.close()
    Tn, ost = oracle.pcg(mesh, o["diag_b"], o["upper"], o["source_b"], p.T0, tol=synth.TOL,
                         rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER)
    assert max_rel(T, Tn) <= 1e-8
    assert abs(st[0]["n_iter"] - ost["n_iter"]) <= 1


@pytest.mark.parametrize("name,mesh,pc", [MESHES[0], MESHES[1], MESHES[2]], ids=IDS[:3])
def test_nonorth_corrector_passes(L, oracle, name, mesh, pc):
    """Two extra passes of the corrector loop per step: the same passes as the
    oracle's (ddt from T at the step's start, correction from the latest T)."""
    m, P = _problem(L, mesh, pc, n_nonorth_corr=2)
    T0 = synth.initial_field(mesh.n_cells, 12)
    P.set_T(T0)
    steps = 3
    _, ostats, osnaps = oracle.run_nonorth(mesh, BCS, DT, dt, steps, T0, n_corr=2,
                                           pc=oracle.PC_DIC if pc == "dic" else oracle.PC_DIAGONAL)
    for s in range(steps):
        st, _ = P.step(1)
        T = P.get_T()
        assert max_rel(T, osnaps[s]) <= 1e-8, (name, s, max_rel(T, osnaps[s]))
        assert abs(st[0]["n_iter"] - ostats[s]["n_iter"]) <= 3, (name, s)
    # the test hook still assembles from the current T (no stale start-of-step copy)
    P.assemble()
    g = P.matrix()
    Tn = P.get_T()
    o = oracle.assemble(mesh, BCS, DT, dt, Tn, lap_src=oracle.step_source(mesh, BCS, DT, Tn))
    assert np.array_equal(g["source"], o["source"])
    P.close()
    m.close()


def test_nonorth_corrector_passes_mixed(L, oracle):
    mesh = synth.affine(synth.box_mesh(12, 10, 8, z_ratio=3.0), synth.SKEW)
    m, P = _problem(L, mesh, "diagonal", precision=L.LF_PREC_MIXED, n_nonorth_corr=1)
    T = synth.initial_field(mesh.n_cells, 13)
    P.set_T(T)
    for s in range(2):
        P.step(1)
        Tg = P.get_T()
        To, _, _ = oracle.run_nonorth(mesh, BCS, DT, dt, 1, T, n_corr=1)
        assert max_rel(Tg, To) <= 1e-8, (s, max_rel(Tg, To))
        T = Tg
    P.close()
    m.close()


def test_corrector_option_checked(L):
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        _problem(L, MESHES[0][1], "diagonal", n_nonorth_corr=-1)


def test_nonorth_rows_layout_on_band_mesh(L, oracle):
    """A band-form mesh solved in the row layout: the correction (taken from
    the mesh's band records) and the assembly (rows) together, bit for bit."""
    mesh = MESHES[0][1]
    m, P = _problem(L, mesh, "diagonal", layout=L.LF_LAYOUT_ROWS)
    assert P.layout() == L.LF_LAYOUT_ROWS
    T0 = synth.initial_field(mesh.n_cells, 14)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, BCS, DT, dt, T0, lap_src=oracle.step_source(mesh, BCS, DT, T0))
    for k in ("diag", "upper", "source", "diag_b", "source_b"):
        assert np.array_equal(g[k], o[k]), k
    st, _ = P.step(2)
    _, ostats, osnaps = oracle.run_nonorth(mesh, BCS, DT, dt, 2, T0)
    assert max_rel(P.get_T(), osnaps[-1]) <= 1e-8
    P.close()
    m.close()
