"""Pins of the oracle's aggregation multigrid preconditioner (no GPU).

Each pin is a plain function of the oracle module (test_oracle_mutants.py runs
them against oracles with planted mistakes):
  - the Galerkin coarse matrix equals P^T A P formed densely (a library matrix
    product), for the box's 2x2x2 aggregation and for an arbitrary one;
  - with one level and one sweep the cycle is omega D^-1 (closed form);
  - with no smoothing and an exact coarse solve the two-level cycle is
    P A_c^-1 P^T, so M A fixes every piecewise-constant vector P v_c;
  - with nu sweeps and an exact coarse solve it is (I - E) A^-1 with the
    textbook two-grid error propagation E = S^nu (I - P A_c^-1 P^T A) S^nu,
    S = I - omega D^-1 A;
  - the cycle is a symmetric positive definite operator (as PCG needs);
  - PCG with it reaches numpy's LU solution, in fewer iterations than with the
    diagonal preconditioner.
"""
import numpy as np

import synth
from tests.helpers import ldu_to_dense


def _system(shape=(6, 5, 4), ratio=3.0, DT=0.05, dt=0.01, seed=3):
    from oracle import oracle as O0     # geometry and assembly only (pinned elsewhere)
    mesh = synth.box_mesh(*shape, z_ratio=ratio)
    T0 = synth.initial_field(mesh.n_cells, seed)
    A = O0.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    return mesh, A["diag_b"], A["upper"], A["source_b"], T0


def _dense_P(agg, nc):
    P = np.zeros((len(agg), nc))
    P[np.arange(len(agg)), agg] = 1.0
    return P


def _cycle_matrix(O, mesh, diag, upper, lc, ag, **kw):
    N = mesh.n_cells
    M = np.empty((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        M[:, i] = O.amg_apply(mesh, diag, upper, e, lc, ag, **kw)
    return M


def pin_galerkin_is_ptap(O):
    mesh, diag, upper, _, _ = _system()
    A = ldu_to_dense(mesh, diag, upper)
    lc, ag = synth.box_aggregation(mesh.shape, coarsest=8)
    rng = np.random.default_rng(1)
    for agg, nc in ((ag[0], lc[1]), (rng.integers(0, 17, mesh.n_cells).astype(np.int32), 17)):
        nc = int(max(nc, agg.max() + 1))
        co, cn, cd, cu = O.galerkin(mesh.n_cells, mesh.owner, mesh.neighbour, diag, upper, agg, nc)
        assert np.all(co < cn)
        key = co.astype(np.int64) * nc + cn
        assert np.all(np.diff(key) > 0)                 # upper-triangular order
        P = _dense_P(agg, nc)
        want = P.T @ A @ P
        got = np.diag(cd)
        got[co, cn] = cu
        got[cn, co] = cu
        assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))
        assert np.count_nonzero(np.triu(want, 1)) == len(cu)


def pin_single_level_is_scaled_jacobi(O):
    mesh, diag, upper, b, _ = _system()
    w = O.amg_apply(mesh, diag, upper, b, [mesh.n_cells], [], nu=0, nu_c=1, omega=0.8)
    assert np.array_equal(w, 0.0 + 0.8 * ((b - 0.0) / diag))


def pin_coarse_correction_is_projection(O):
    """nu = 0, coarse solve by many sweeps: M = P A_c^-1 P^T, so M A P v = P v."""
    mesh, diag, upper, _, _ = _system()
    lc, ag = synth.box_aggregation(mesh.shape, coarsest=30)
    assert len(lc) == 2
    A = ldu_to_dense(mesh, diag, upper)
    P = _dense_P(ag[0], lc[1])
    v = P @ np.random.default_rng(2).uniform(-1, 1, lc[1])
    got = O.amg_apply(mesh, diag, upper, A @ v, lc, ag, nu=0, nu_c=3000)
    assert np.max(np.abs(got - v)) <= 1e-10 * np.max(np.abs(v))


def pin_two_grid_operator(O):
    """Two levels, nu = 2 sweeps, an exact coarse solve: M = (I - E) A^-1."""
    mesh, diag, upper, _, _ = _system()
    lc, ag = synth.box_aggregation(mesh.shape, coarsest=30)
    A = ldu_to_dense(mesh, diag, upper)
    N = mesh.n_cells
    P = _dense_P(ag[0], lc[1])
    Ac = P.T @ A @ P
    S = np.eye(N) - 0.8 * (A / diag[:, None])
    S2 = S @ S
    E = S2 @ (np.eye(N) - P @ np.linalg.solve(Ac, P.T @ A)) @ S2
    want = (np.eye(N) - E) @ np.linalg.inv(A)
    got = _cycle_matrix(O, mesh, diag, upper, lc, ag, nu=2, nu_c=3000, omega=0.8)
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def pin_cycle_is_spd(O):
    mesh, diag, upper, _, _ = _system()
    lc, ag = synth.box_aggregation(mesh.shape, coarsest=8, min_side=2)
    assert len(lc) == 3
    M = _cycle_matrix(O, mesh, diag, upper, lc, ag)
    assert np.max(np.abs(M - M.T)) <= 1e-13 * np.max(np.abs(M))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0.0


def pin_pcg_reaches_lu(O):
    mesh, diag, upper, b, T0 = _system(shape=(12, 11, 10), ratio=5.0, DT=0.5, dt=0.01)
    A = ldu_to_dense(mesh, diag, upper)
    exact = np.linalg.solve(A, b)
    lc, ag = synth.box_aggregation(mesh.shape, coarsest=20)
    assert len(lc) >= 3
    x, st = O.pcg_amg(mesh, diag, upper, b, T0, lc, ag, tol=1e-14)
    assert np.max(np.abs(x - exact) / np.abs(exact)) <= 1e-11
    _, sa = O.pcg_amg(mesh, diag, upper, b, T0, lc, ag, tol=1e-9)
    _, sd = O.pcg(mesh, diag, upper, b, T0, tol=1e-9)
    assert sa["converged"] == 1 and sa["final_residual"] < 1e-9
    assert sa["n_iter"] < sd["n_iter"], (sa["n_iter"], sd["n_iter"])


PINS = [pin_galerkin_is_ptap, pin_single_level_is_scaled_jacobi, pin_coarse_correction_is_projection,
        pin_two_grid_operator, pin_cycle_is_spd, pin_pcg_reaches_lu]


def test_galerkin_is_ptap(oracle):
    pin_galerkin_is_ptap(oracle)


def test_single_level_is_scaled_jacobi(oracle):
    pin_single_level_is_scaled_jacobi(oracle)


def test_coarse_correction_is_projection(oracle):
    pin_coarse_correction_is_projection(oracle)


def test_two_grid_operator(oracle):
    pin_two_grid_operator(oracle)


def test_cycle_is_spd(oracle):
    pin_cycle_is_spd(oracle)


def test_pcg_reaches_lu(oracle):
    pin_pcg_reaches_lu(oracle)


def test_box_aggregation_blocks():
    """Each aggregate of the box hierarchy is a block of at most 2 cells per
    direction, numbered on the halved box; odd lengths end with a one-cell block."""
    shape = (7, 4, 3)
    lc, ag = synth.box_aggregation(shape, coarsest=1, min_side=1)
    assert lc == [84, 16, 2, 1] and len(ag) == 3
    nx, ny, nz = shape
    c = np.arange(nx * ny * nz)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    cx, cy = (nx + 1) // 2, (ny + 1) // 2
    assert np.array_equal(ag[0], i // 2 + cx * (j // 2 + cy * (k // 2)))
    assert np.bincount(ag[0]).tolist().count(8) == 3 * 2 * 1
    # the default keeps every level a box of sides >= 2 and stops at 512 cells
    assert synth.box_aggregation((256, 256, 256))[0] == [256 ** 3, 128 ** 3, 64 ** 3, 32 ** 3, 16 ** 3, 8 ** 3]
    assert synth.box_aggregation((100, 100, 100))[0] == [100 ** 3, 50 ** 3, 25 ** 3, 13 ** 3, 7 ** 3]
    assert synth.box_aggregation((40, 5, 4))[0] == [800, 3 * 20 * 2]
