"""Precision form (FP32 inner CG on the Jacobi-scaled system with FP64 dots /
alpha / beta, FP64 outer refinement on the true residual) against the FP64
oracle.

Per step, both solve the same system: the oracle takes one step from the
precision form's own T_n, and T_{n+1} must agree to a max relative error of
1e-8.  (Trajectories of two different solvers that each stop below the
tolerance drift apart by more than that over many steps: the oracle's own
trajectory at tol 1e-9 is 1.3e-8 away from the exactly solved one after 20
steps of the 32^3 case.)  The FP64 true residual of every result, recomputed
on the host from the oracle's matrix, is below the tolerance."""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam, run_gpu, max_rel
from tests.helpers import norm_factor, ldu_to_dense

pytestmark = pytest.mark.gpu

T_TOL = 1e-8


@pytest.fixture(scope="module")
def L():
    return lapfoam()


CASES = [
    ("plain_32", "plain_32", None, 20, {}),
    ("graded_24", "graded_256", 24, 6, {}),
    ("permuted_20", "permuted_192", 20, 6, {}),
    ("graded_24_loose_inner", "graded_256", 24, 4, dict(inner_tol=1e-2)),
    ("graded_24_tight_inner", "graded_256", 24, 4, dict(inner_tol=1e-6)),
    ("graded_24_no_graph", "graded_256", 24, 3, dict(use_graph=0)),
    ("graded_24_walk", "graded_256", 24, 4, dict(amul_walk=1)),
    ("graded_13_walk_rows", "graded_256", 13, 4, dict(amul_walk=1, layout=1)),
    ("plain_32_walk", "plain_32", None, 6, dict(amul_walk=1)),
    # nx = 18: the FP64 products by the block walk, the FP32 ones by the row walk
    ("graded_18_walk", "graded_256", 18, 4, dict(amul_walk=1)),
    ("graded_20_walk", "graded_256", 20, 4, dict(amul_walk=1)),
    ("graded_24_restart", "graded_256", 24, 4, dict(inner_restart=1)),
    ("permuted_20_restart", "permuted_192", 20, 4, dict(inner_restart=1)),
    ("graded_24_tight_continued", "graded_256", 24, 4, dict(inner_tol=1e-3)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mixed_matches_fp64_oracle(L, oracle, case):
    name, cfg, n, steps, extra = case
    p = synth.build_config(cfg, n=n, steps=steps)
    Tg, sg = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, steps, precision=L.LF_PREC_MIXED, **extra)
    To, so, snaps = oracle.run(p.mesh, p.bcs, p.DT, p.dt, steps, p.T0, keep_all=True)
    T_prev = p.T0
    for s in range(steps):
        ref, _, _ = oracle.run(p.mesh, p.bcs, p.DT, p.dt, 1, T_prev)
        err = max_rel(Tg[s], ref)
        assert err <= T_TOL, (s, err)
        assert sg[s]["converged"] == 1 and sg[s]["final_residual"] < 1e-9
        assert sg[s]["n_outer"] >= 1
        # step 1 starts from the same T0 as the oracle; later steps start from
        # a T that differs at the solver-tolerance level
        rtol = 1e-10 if s == 0 else 1e-6
        assert abs(sg[s]["initial_residual"] - so[s]["initial_residual"]) <= \
            rtol * so[s]["initial_residual"]
        # the FP64 true residual of the GPU result, from the oracle's matrix
        m = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, T_prev)
        r = m["source_b"] - oracle.amul(p.mesh, m["diag_b"], m["upper"], Tg[s])
        A1 = oracle.sum_a(p.mesh, m["diag_b"], m["upper"])
        Ax0 = oracle.amul(p.mesh, m["diag_b"], m["upper"], T_prev)
        pA = A1 * T_prev.mean()
        nf = np.sum(np.abs(Ax0 - pA) + np.abs(m["source_b"] - pA)) + 1e-20
        assert np.sum(np.abs(r)) / nf < 1e-9 * (1 + 1e-6)
        T_prev = Tg[s]      # the system of the next step is built from the GPU field


def test_mixed_is_deterministic(L):
    p = synth.build_config("permuted_192", n=18, steps=3)
    a, sa = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 3, precision=L.LF_PREC_MIXED)
    b, sb = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 3, precision=L.LF_PREC_MIXED,
                    iters_per_check=1)
    for s in range(3):
        assert np.array_equal(a[s], b[s])
        assert sa[s]["n_iter"] == sb[s]["n_iter"] and sa[s]["n_outer"] == sb[s]["n_outer"]


def test_mixed_edge_cases(L, oracle):
    # zero diffusivity: converged at the start, no pass
    mesh = synth.box_mesh(6, 6, 6)
    T0 = synth.initial_field(mesh.n_cells, 3)
    Tg, sg = run_gpu(L, mesh, synth.fixed_x_bcs(), 0.0, 1e-3, T0, 2, precision=L.LF_PREC_MIXED)
    assert all(s["n_iter"] == 0 and s["n_outer"] == 0 and s["converged"] == 1 for s in sg)
    # one cell, and a line
    for mesh in (synth.box_mesh(1, 1, 1), synth.box_mesh(17, 1, 1)):
        T0 = synth.initial_field(mesh.n_cells, 4)
        Tg, sg = run_gpu(L, mesh, synth.fixed_x_bcs(), 0.3, 0.2, T0, 2, precision=L.LF_PREC_MIXED)
        To, so, snaps = oracle.run(mesh, synth.fixed_x_bcs(), 0.3, 0.2, 2, T0, keep_all=True)
        assert max_rel(Tg[0], snaps[0]) <= T_TOL
    # refinement cap: one pass only, so it stops unconverged but finite
    p = synth.build_config("graded_256", n=12, steps=1)
    Tg, sg = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 1, precision=L.LF_PREC_MIXED,
                     max_outer=1, inner_tol=0.5)
    assert sg[0]["n_outer"] == 1 and sg[0]["converged"] == 0
    assert np.all(np.isfinite(Tg[0]))


def test_mixed_refuses_dic(L):
    mesh = synth.renumber(synth.box_mesh(4, 4, 4),
                          synth.red_black_numbering(synth.box_mesh(4, 4, 4))[0])
    m = L.Mesh(mesh)
    with pytest.raises(L.LapfoamError):
        L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3,
                  L.make_opts(precond=L.LF_PC_DIC, precision=L.LF_PREC_MIXED))
    m.close()


INNER_MESHES = [
    # (name, mesh, expected product form under LF_WALK_ON; FP32 block walk when nx % 4 == 0)
    ("box_132x7x5", lambda: synth.box_mesh(132, 7, 5, z_ratio=3.0), 2),     # tiles cross waves, odd lines/planes
    ("box_4x9x3", lambda: synth.box_mesh(4, 9, 3), 2),                      # one thread per tile line
    ("box_256x2x3", lambda: synth.box_mesh(256, 2, 3, z_ratio=2.0), 2),     # one wave per tile line
    ("box_18x5x4", lambda: synth.box_mesh(18, 5, 4), 2),                    # FP64 block walk, FP32 row walk
    ("box_13x6x5", lambda: synth.box_mesh(13, 6, 5), 1),                    # row walk
]


@pytest.mark.parametrize("name,mk,form", INNER_MESHES, ids=[c[0] for c in INNER_MESHES])
def test_inner_product_forms_bitwise(L, name, mk, form):
    """The inner FP32 product in the walk forms equals the one-row-per-thread
    product bitwise (the FP32 coefficients do not depend on T, so one step of
    each problem forms the same ones)."""
    import torch
    mesh = mk()
    T0 = synth.initial_field(mesh.n_cells, 17)
    x = torch.from_numpy(np.random.default_rng(5).uniform(-1.0, 1.0, mesh.n_cells).astype(np.float32)).cuda()
    m = L.Mesh(mesh)
    ys = []
    for walk in (L.LF_WALK_ON, L.LF_WALK_OFF):
        P = L.Problem(m, synth.fixed_x_bcs(), 2e-3, 1e-3,
                      L.make_opts(amul_walk=walk, precision=L.LF_PREC_MIXED))
        assert P.amul_form() == (form if walk == L.LF_WALK_ON else 0)
        with pytest.raises(L.LapfoamError, match="LF_ESTATE"):
            P.amul_inner(x, torch.empty_like(x))
        P.set_T(T0)
        P.step(1)
        y = torch.full_like(x, float("nan"))
        P.amul_inner(x, y)
        torch.cuda.synchronize()
        ys.append(y.cpu().numpy())
        P.close()
    assert np.array_equal(ys[0], ys[1]), name
    assert np.all(np.isfinite(ys[0]))
    m.close()
