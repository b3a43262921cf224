"""Parity at the full sizes of the timed workloads, in the launch configuration
the benchmark times (default options: iteration blocks captured as graphs,
adaptive convergence checks, several time steps in one call).

At these sizes the oracle still finishes a time step in seconds, so every
output is compared, not a sample: the assembled coefficients and one LDU
product bitwise, T after each step within 1e-8 (max relative) of the oracle's
solve of the same system, iteration counts within one.
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


def _problem(L, p, precision=None):
    precond = L.LF_PC_DIC if p.precond == "dic" else L.LF_PC_DIAGONAL
    if precision is None:
        precision = L.LF_PREC_MIXED if p.precision == "mixed" else L.LF_PREC_FP64
    opts = L.make_opts(tol=synth.TOL, rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER,
                       precond=precond, precision=precision)
    m = L.Mesh(p.mesh)
    return m, L.Problem(m, p.bcs, p.DT, p.dt, opts), precond


@pytest.mark.parametrize("cfg", ["graded_256", "permuted_192"])
def test_full_size_matrix_and_amul_bitwise(L, oracle, cfg):
    import torch
    p = synth.build_config(cfg)
    m, P, _ = _problem(L, p)
    # the 256^3 band layout takes the row-walk product by default (the
    # configuration the benchmark times); the permuted mesh has no band form
    assert P.amul_walk() == (cfg == "graded_256")
    P.set_T(p.T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, p.T0)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        assert np.array_equal(g[k], o[k]), k
    x = np.random.default_rng(11).uniform(-1.0, 1.0, p.mesh.n_cells)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    P.amul(xd, yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), oracle.amul(p.mesh, o["diag_b"], o["upper"], x))
    P.close()
    m.close()


@pytest.mark.parametrize("cfg,steps", [("graded_256", 2), ("permuted_192", 2), ("graded_256_dic", 1)])
def test_full_size_steps_match_oracle(L, oracle, cfg, steps):
    p = synth.build_config(cfg, steps=steps)
    m, P, pc = _problem(L, p)
    # the forms the benchmark times: the block walk with the solve on the
    # Jacobi-scaled matrix, one row per thread on the row layout, DIC's
    # kernels with two red-black pairs per lane on the two-colour layout
    assert P.amul_form() == {"graded_256": 4, "permuted_192": 0, "graded_256_dic": 3}[cfg]
    P.set_T(p.T0)
    sg, _ = P.step(steps)                  # one call for all steps, as the benchmark does
    Tg = P.get_T()
    P.close()
    m.close()
    To, so, _ = oracle.run(p.mesh, p.bcs, p.DT, p.dt, steps, p.T0, pc=pc)
    assert max_rel(Tg, To) <= T_TOL, max_rel(Tg, To)
    for s in range(steps):
        assert abs(sg[s]["n_iter"] - so[s]["n_iter"]) <= 1, (s, sg[s], so[s])
        assert sg[s]["converged"] == 1 and so[s]["converged"] == 1
        assert abs(sg[s]["initial_residual"] - so[s]["initial_residual"]) <= \
            1e-10 * so[s]["initial_residual"]
        assert sg[s]["final_residual"] < synth.TOL


def _paper_box(n):
    """One of the paper's evaluation boxes: uniform n^3 cells on the unit cube,
    DT = 1e-4 (unstated in the paper), dt = 0.2, the configs' boundary
    conditions and T0 recipe."""
    return synth.box_mesh(n, n, n), synth.fixed_x_bcs(), 1e-4, 0.2, \
        synth.initial_field(n ** 3, 20250724)


def test_paper_shape_100_steps_match_oracle(L, oracle):
    """Mesh-S (100^3) at the paper's time step: five steps in the benchmark's
    launch configuration, each against the oracle's step from the same T."""
    mesh, bcs, DT, dt, T0 = _paper_box(100)
    m = L.Mesh(mesh)
    P = L.Problem(m, bcs, DT, dt, L.make_opts(tol=synth.TOL))
    P.set_T(T0)
    T_prev = T0
    for s in range(5):
        sg, _ = P.step(1)
        Tg = P.get_T()
        To, so, _ = oracle.run(mesh, bcs, DT, dt, 1, T_prev)
        assert max_rel(Tg, To) <= T_TOL, (s, max_rel(Tg, To))
        assert abs(sg[0]["n_iter"] - so[0]["n_iter"]) <= 1, (s, sg[0], so[0])
        assert sg[0]["converged"] == 1 and so[0]["converged"] == 1
        T_prev = Tg
    P.close()
    m.close()


def test_paper_shape_300_one_step(L, oracle):
    """Mesh-L (300^3, 27 M cells, 80.7 M internal faces), the largest size
    compared with the oracle: the matrix bitwise, one time step within 1e-8."""
    mesh, bcs, DT, dt, T0 = _paper_box(300)
    m = L.Mesh(mesh)
    P = L.Problem(m, bcs, DT, dt, L.make_opts(tol=synth.TOL))
    assert P.layout() == L.LF_LAYOUT_BANDS and P.amul_walk()
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, bcs, DT, dt, T0)
    for k in ("diag", "upper", "source", "diag_b", "source_b"):
        assert np.array_equal(g[k], o[k]), k
    del g, o
    sg, _ = P.step(1)
    Tg = P.get_T()
    P.close()
    m.close()
    To, so, _ = oracle.run(mesh, bcs, DT, dt, 1, T0)
    assert max_rel(Tg, To) <= T_TOL, max_rel(Tg, To)
    assert abs(sg[0]["n_iter"] - so[0]["n_iter"]) <= 1, (sg[0], so[0])


def test_full_size_mixed_twenty_steps(L, oracle):
    """The precision form over the benchmark's 20 steps of the 256^3 box, each
    step on the same system (from the precision form's own T_n): within 1e-8 of
    an FP64 solve of that system converged to tol 1e-13 on the GPU at every
    step, and of the oracle's converged solve at steps 1, 2 and 20 (which also
    pins the GPU's converged solve); the stopping residual below tol."""
    import torch
    p = synth.build_config("mixed_256", steps=20)
    m, P, _ = _problem(L, p)
    R = L.Problem(m, p.bcs, p.DT, p.dt, L.make_opts(tol=1e-13, rel_tol=0.0, max_iter=synth.MAX_ITER))
    N = p.mesh.n_cells
    a = torch.from_numpy(p.T0).cuda()
    t = torch.empty_like(a)
    P.set_T(a)
    for s in range(20):
        T_prev = a.clone()
        R.set_T(T_prev)
        sg, _ = P.step(1)
        R.step(1)
        P.get_T(a)
        R.get_T(t)
        err = float(((a - t).abs() / t.abs()).max())
        assert err <= T_TOL, (s, err)
        assert sg[0]["converged"] == 1 and sg[0]["final_residual"] < synth.TOL
        if s in (0, 1, 19):
            exact, _, _ = oracle.run(p.mesh, p.bcs, p.DT, p.dt, 1, T_prev.cpu().numpy(), tol=1e-13)
            Tg = a.cpu().numpy()
            assert max_rel(Tg, exact) <= T_TOL, (s, max_rel(Tg, exact))
            assert max_rel(t.cpu().numpy(), exact) <= 1e-10, s
    assert a.numel() == N
    R.close()
    P.close()
    m.close()
