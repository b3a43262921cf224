"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

Each test would fail for a plausible slip in the oracle: a dropped or
mis-signed boundary term, a transposed owner/neighbour, a wrong time-term
factor, a wrong residual normalisation or a broken CG recurrence.
"""
import math

import numpy as np
import pytest

import synth
from synth import FIXED_VALUE, ZERO_GRADIENT
from tests.helpers import stencil_system, ldu_to_dense, norm_factor, line_mesh

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

BCS = synth.fixed_x_bcs()
ZG = synth.all_zero_gradient()


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# --------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,ratio,numbering", [
    ((4, 4, 4), 1.0, "natural"), ((3, 2, 5), 4.0, "natural"), ((4, 3, 4), 10.0, "random"),
    ((4, 4, 2), 2.0, "red_black")])
def test_assembly_matches_dense_stencil(oracle, shape, ratio, numbering):
    """Oracle LDU scattered to dense equals an independent (i,j,k) stencil."""
    mesh = synth.box_mesh(*shape, z_ratio=ratio)
    if numbering == "random":
        mesh = synth.renumber(mesh, synth.random_permutation(mesh.n_cells, 3))
    elif numbering == "red_black":
        mesh = synth.renumber(mesh, synth.red_black_numbering(mesh)[0])
    T = synth.initial_field(mesh.n_cells, 11)
    DT, dt = 0.37, 0.05
    bcs = [(FIXED_VALUE, 273.0), (FIXED_VALUE, 573.0), (ZERO_GRADIENT, 0.0),
           (FIXED_VALUE, 400.0), (ZERO_GRADIENT, 0.0), (ZERO_GRADIENT, 0.0)]
    m = oracle.assemble(mesh, bcs, DT, dt, T)
    A = ldu_to_dense(mesh, m["diag_b"], m["upper"])
    A_ref, b_ref = stencil_system(mesh, bcs, DT, dt, T)
    assert _rel(A, A_ref) < 1e-14
    assert _rel(m["source_b"], b_ref) < 1e-14
    # without the boundary: diag/source exclude the fixedValue contributions
    Ab = ldu_to_dense(mesh, m["diag"], m["upper"])
    assert np.all(np.diag(Ab) <= np.diag(A) + 1e-300)
    V = mesh.cell_volume
    assert _rel(m["source"], V / dt * T) < 1e-15


@pytest.mark.parametrize("name", ["plain_32", "graded_256", "permuted_192", "graded_256_dic"])
def test_matrix_invariants(oracle, name):
    """Symmetric LDU, negative off-diagonals, row sums, strict dominance."""
    p = synth.build_config(name, n=12)
    m = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, p.T0)
    assert np.all(m["upper"] < 0)
    assert np.all(m["diag_b"] > 0)
    # row sum of A = V/dt + sum of fixedValue internal coefficients of the cell
    row = m["diag_b"].copy()
    np.add.at(row, p.mesh.owner, m["upper"])
    np.add.at(row, p.mesh.neighbour, m["upper"])
    expect = p.mesh.cell_volume / p.dt
    np.add.at(expect, p.mesh.bface_cell, m["int_coeff"])
    assert _rel(row, expect) < 1e-12
    # strict diagonal dominance: diag - sum|offdiag| = V/dt + boundary > 0
    off = np.zeros(p.mesh.n_cells)
    np.add.at(off, p.mesh.owner, np.abs(m["upper"]))
    np.add.at(off, p.mesh.neighbour, np.abs(m["upper"]))
    assert np.all(m["diag_b"] - off > 0)
    # boundary coefficients only on the two fixedValue patches
    ps = p.mesh.patch_start
    assert np.all(m["int_coeff"][ps[0]:ps[2]] > 0)
    assert np.all(m["int_coeff"][ps[2]:] == 0) and np.all(m["bou_coeff"][ps[2]:] == 0)
    # the oracle's own row sums agree with the definition
    assert _rel(oracle.sum_a(p.mesh, m["diag_b"], m["upper"]), row) < 1e-14


def test_amul_against_dense(oracle):
    mesh = synth.renumber(synth.box_mesh(5, 4, 3, z_ratio=3.0),
                          synth.random_permutation(60, 5))
    rng = np.random.default_rng(0)
    diag = rng.uniform(1, 2, mesh.n_cells)
    upper = rng.uniform(-1, 0, mesh.n_faces)
    x = rng.uniform(-1, 1, mesh.n_cells)
    y = oracle.amul(mesh, diag, upper, x)
    A = ldu_to_dense(mesh, diag, upper)
    assert _rel(y, A @ x) < 1e-14


# --------------------------------------------------------------------------
# solve
# --------------------------------------------------------------------------
def test_pcg_matches_lu_4cubed(oracle):
    """PCG at tight tolerance reproduces numpy/LAPACK's LU solve."""
    p = synth.build_config("plain_32", n=4)
    m = oracle.assemble(p.mesh, p.bcs, 0.05, 0.2, p.T0)
    A = ldu_to_dense(p.mesh, m["diag_b"], m["upper"])
    x_lu = np.linalg.solve(A, m["source_b"])
    for pc in (oracle.PC_DIAGONAL, oracle.PC_DIC):
        x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, pc=pc,
                           tol=1e-14)
        assert st["converged"] == 1
        assert _rel(x, x_lu) < 1e-12


def test_one_cell_closed_form(oracle):
    mesh = synth.box_mesh(1, 1, 1, lengths=(0.5, 0.25, 2.0))
    DT, dt, T0 = 0.7, 0.3, np.array([350.0])
    T, st, _ = oracle.run(mesh, BCS, DT, dt, 1, T0, tol=1e-15)
    V = 0.5 * 0.25 * 2.0
    cb = DT * (0.25 * 2.0) / 0.25          # area / half-width, each x wall
    expect = (V / dt * 350.0 + cb * 273.0 + cb * 573.0) / (V / dt + 2 * cb)
    assert abs(T[0] - expect) <= 1e-13 * expect


def test_two_cell_closed_form(oracle):
    mesh = synth.box_mesh(2, 1, 1)
    DT, dt = 0.2, 0.1
    T0 = np.array([300.0, 500.0])
    T, st, _ = oracle.run(mesh, BCS, DT, dt, 1, T0, tol=1e-15)
    V = 0.5
    c = DT * 1.0 / 0.5        # interior: area 1, centre distance 0.5
    cb = DT * 1.0 / 0.25      # wall: area 1, half width 0.25
    a11 = a22 = V / dt + c + cb
    b1, b2 = V / dt * 300.0 + cb * 273.0, V / dt * 500.0 + cb * 573.0
    det = a11 * a22 - c * c
    x1, x2 = (b1 * a22 + c * b2) / det, (a11 * b2 + c * b1) / det
    assert abs(T[0] - x1) <= 1e-13 * x1 and abs(T[1] - x2) <= 1e-13 * x2


@pytest.mark.parametrize("ratio", [1.0, 10.0])
def test_steady_linear_profile(oracle, ratio):
    """A huge time step gives the exact linear steady state 273 + 300 x."""
    mesh = synth.box_mesh(12, 5, 6, z_ratio=ratio)
    T0 = synth.initial_field(mesh.n_cells, 4)
    T, st, _ = oracle.run(mesh, BCS, 1.0, 1e30, 1, T0, tol=1e-14)
    exact = 273.0 + 300.0 * mesh.cell_centre[:, 0]
    assert st[0]["converged"] == 1
    assert _rel(T, exact) < 1e-11


def test_cosine_mode_exact_discrete_decay(oracle):
    """With zeroGradient walls cos(pi x) is an eigenvector of the two-point
    Laplacian on uniform cells, eigenvalue (4/dx^2) sin^2(pi dx/2); each implicit
    Euler step multiplies it by 1/(1 + dt DT lambda)."""
    n = 16
    mesh = synth.box_mesh(n, 3, 2)
    DT, dt, A0, B0 = 0.02, 0.3, 400.0, 50.0
    x = mesh.cell_centre[:, 0]
    T0 = A0 + B0 * np.cos(math.pi * x)
    dx = 1.0 / n
    lam = 4.0 / dx ** 2 * math.sin(math.pi * dx / 2) ** 2
    g = 1.0 / (1.0 + dt * DT * lam)
    T, st, snaps = oracle.run(mesh, ZG, DT, dt, 3, T0, tol=1e-15, keep_all=True)
    for s, Ts in enumerate(snaps, start=1):
        expect = A0 + B0 * g ** s * np.cos(math.pi * x)
        assert np.max(np.abs(Ts - expect)) < 1e-10


def test_sine_mode_second_order_convergence(oracle):
    """T0 = 273 + 300x + B sin(pi x) with fixed x walls decays as
    exp(-DT pi^2 t); the error falls ~4x when dx halves and dt quarters."""
    DT, B, t_end = 1.0, 50.0, 0.05
    errs = []
    for n in (8, 16, 32, 64):
        mesh = line_mesh(n)
        x = mesh.cell_centre[:, 0]
        steps = n * n // 4
        dt = t_end / steps
        T0 = 273.0 + 300.0 * x + B * np.sin(math.pi * x)
        T, st, _ = oracle.run(mesh, BCS, DT, dt, steps, T0, tol=1e-14)
        exact = 273.0 + 300.0 * x + B * math.exp(-DT * math.pi ** 2 * t_end) * np.sin(math.pi * x)
        errs.append(np.max(np.abs(T - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.5 < r < 4.5 for r in ratios), (errs, ratios)


def test_heat_conservation_all_zero_gradient(oracle):
    """Columns of A sum to V/dt, so sum V (T1 - T0) = -dt * sum(b - A T1)."""
    p = synth.build_config("graded_256", n=10)
    T0 = p.T0
    DT, dt = 1e-3, 1e-3
    T1, st, _ = oracle.run(p.mesh, ZG, DT, dt, 1, T0)
    m = oracle.assemble(p.mesh, ZG, DT, dt, T0)
    A = ldu_to_dense(p.mesh, m["diag_b"], m["upper"])
    r = m["source_b"] - A @ T1
    V = p.mesh.cell_volume
    lhs = abs(np.sum(V * T1) - np.sum(V * T0))
    slack = 64 * np.finfo(float).eps * np.sum(V * np.abs(T0))
    assert lhs <= dt * np.sum(np.abs(r)) + slack
    assert st[0]["n_iter"] > 0


# --------------------------------------------------------------------------
# PCG semantics
# --------------------------------------------------------------------------
def test_zero_diffusivity_needs_no_iteration(oracle):
    p = synth.build_config("plain_32", n=6)
    T, st, _ = oracle.run(p.mesh, ZG, 0.0, 1e-3, 2, p.T0)
    assert all(s["n_iter"] == 0 and s["converged"] == 1 for s in st)
    assert _rel(T, p.T0) < 1e-15


def test_diagonal_matrix_one_iteration(oracle):
    p = synth.build_config("plain_32", n=5)
    rng = np.random.default_rng(2)
    diag = rng.uniform(1, 3, p.mesh.n_cells)
    upper = np.zeros(p.mesh.n_faces)
    b = rng.uniform(-1, 1, p.mesh.n_cells)
    x, st = oracle.pcg(p.mesh, diag, upper, b, np.zeros(p.mesh.n_cells), tol=1e-12)
    assert st["n_iter"] == 1 and st["converged"] == 1
    assert _rel(x, b / diag) < 1e-15


def test_error_a_norm_monotone_and_true_residual(oracle):
    p = synth.build_config("graded_256", n=5)
    m = oracle.assemble(p.mesh, p.bcs, 0.05, 0.05, p.T0)
    A = ldu_to_dense(p.mesh, m["diag_b"], m["upper"])
    b = m["source_b"]
    x_star = np.linalg.solve(A, b)
    nf = norm_factor(A, b, p.T0)
    prev = np.inf
    for k in range(1, 12):
        x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], b, p.T0, tol=0.0, max_iter=k)
        assert st["n_iter"] == k
        e = x - x_star
        ea = math.sqrt(e @ A @ e)
        assert ea <= prev * (1 + 1e-12) + 1e-12
        prev = ea
        true_res = np.sum(np.abs(b - A @ x)) / nf
        assert abs(true_res - st["final_residual"]) <= 1e-12 + 1e-6 * true_res
    x0_res = np.sum(np.abs(b - A @ p.T0)) / nf
    assert abs(st["initial_residual"] - x0_res) <= 1e-14 * x0_res


def test_max_iter_semantics(oracle):
    """The convergence check is skipped once maxIter is reached."""
    p = synth.build_config("plain_32", n=6)
    m = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, p.T0)
    _, st0 = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, max_iter=1,
                        tol=0.0)
    tol = 0.9 * st0["initial_residual"]
    assert st0["final_residual"] < tol
    # one iteration reaches tol, but at maxIter = 1 the check is not made
    x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, max_iter=1,
                       tol=tol)
    assert st["n_iter"] == 1 and st["converged"] == 0
    x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, max_iter=2,
                       tol=tol)
    assert st["n_iter"] == 1 and st["converged"] == 1
    # minIter forces iterations past convergence
    x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, max_iter=50,
                       tol=1.0, min_iter=3)
    assert st["n_iter"] == 3
    x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, tol=1e-9,
                       rel_tol=1e-2)
    assert st["converged"] == 1
    assert st["final_residual"] < 1e-2 * st["initial_residual"]
    x2, st2 = oracle.pcg(p.mesh, m["diag_b"], m["upper"], m["source_b"], p.T0, tol=1e-9)
    assert st2["n_iter"] > st["n_iter"]


def test_singular_break(oracle):
    """A zero right-hand side with x0 = 0 has nothing to do: res0 = 0 < tol."""
    p = synth.build_config("plain_32", n=4)
    m = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, p.T0)
    x, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], np.zeros(p.mesh.n_cells),
                       np.zeros(p.mesh.n_cells), tol=-1.0, max_iter=5)
    # tol < 0 forces the loop: w = 0, wApA = 0 -> singular, no iteration counted
    assert st["singular"] == 1 and st["n_iter"] == 0
    assert np.all(x == 0)


# --------------------------------------------------------------------------
# DIC
# --------------------------------------------------------------------------
def test_dic_exact_on_a_chain(oracle):
    """On a 1-D chain in natural order DIC is the exact Cholesky factor."""
    mesh = line_mesh(40, z_ratio=1.0)
    T0 = synth.initial_field(40, 9)
    m = oracle.assemble(mesh, BCS, 0.5, 0.01, T0)
    x, st = oracle.pcg(mesh, m["diag_b"], m["upper"], m["source_b"], T0,
                       pc=oracle.PC_DIC, tol=1e-13)
    assert st["n_iter"] == 1
    A = ldu_to_dense(mesh, m["diag_b"], m["upper"])
    assert _rel(x, np.linalg.solve(A, m["source_b"])) < 1e-13


def test_dic_matches_factorisation_definition(oracle):
    """rD and the two sweeps equal (D + L) D^-1 (D + L^T) applied by solves."""
    p = synth.build_config("graded_256_dic", n=4)
    m = oracle.assemble(p.mesh, p.bcs, p.DT, p.dt, p.T0)
    rd = oracle.dic_rd(p.mesh, m["diag_b"], m["upper"])
    N = p.mesh.n_cells
    # D_dic from its recurrence written densely, in cell order
    A = ldu_to_dense(p.mesh, m["diag_b"], m["upper"])
    L = np.tril(A, -1)
    d = np.diag(A).copy()
    for c in range(N):
        for l in range(c):
            if L[c, l] != 0:
                d[c] -= L[c, l] ** 2 / d[l]
    assert _rel(1.0 / d, rd) < 1e-14
    r = np.random.default_rng(1).uniform(-1, 1, N)
    w = oracle.precondition(p.mesh, oracle.PC_DIC, m["upper"], rd, r)
    D = np.diag(d)
    M = (D + L) @ np.diag(1.0 / d) @ (D + L.T)
    assert _rel(M @ w, r) < 1e-13


def test_red_black_and_natural_solutions_agree(oracle):
    base = synth.build_config("graded_256", n=8)
    rb = synth.build_config("graded_256_dic", n=8)
    new_of_old, _ = synth.red_black_numbering(base.mesh)
    Tn, stn, _ = oracle.run(base.mesh, base.bcs, base.DT, base.dt, 2, base.T0, tol=1e-13)
    Tr, str_, _ = oracle.run(rb.mesh, rb.bcs, rb.DT, rb.dt, 2, rb.T0, pc=oracle.PC_DIC,
                             tol=1e-13)
    assert _rel(Tr[new_of_old], Tn) < 1e-11
    assert str_[0]["n_iter"] < stn[0]["n_iter"]


@pytest.mark.parametrize("pc", [0, 1])
def test_cg_iterates_are_krylov_optimal(oracle, pc):
    """Iterate k of PCG minimises the A-norm error over x0 + K_k(M^-1 A, M^-1 r0),
    M the preconditioner (diag(A), or (D+L) D^-1 (D+L^T) with D the DIC
    diagonal).  This fixes alpha and beta, not just eventual convergence."""
    p = synth.build_config("graded_256_dic" if pc else "graded_256", n=5)
    m = oracle.assemble(p.mesh, p.bcs, 0.3, 0.02, p.T0)
    A = ldu_to_dense(p.mesh, m["diag_b"], m["upper"])
    b = m["source_b"]
    x0 = p.T0
    x_star = np.linalg.solve(A, b)
    if pc == 0:
        M = np.diag(np.diag(A))
    else:
        d = 1.0 / oracle.dic_rd(p.mesh, m["diag_b"], m["upper"])
        L = np.tril(A, -1)
        M = (np.diag(d) + L) @ np.diag(1.0 / d) @ (np.diag(d) + L.T)
    Minv_A = np.linalg.solve(M, A)
    z = np.linalg.solve(M, b - A @ x0)
    for k in range(1, 6):
        K = np.empty((A.shape[0], k))
        v = z.copy()
        for j in range(k):
            K[:, j] = v
            v = Minv_A @ v
        Q, _ = np.linalg.qr(K)
        y = np.linalg.solve(Q.T @ A @ Q, Q.T @ (A @ (x_star - x0)))
        x_opt = x0 + Q @ y
        xk, st = oracle.pcg(p.mesh, m["diag_b"], m["upper"], b, x0, pc=pc, tol=0.0,
                            max_iter=k)
        assert st["n_iter"] == k
        assert np.max(np.abs(xk - x_opt)) <= 1e-9 * np.max(np.abs(x_star - x0))
