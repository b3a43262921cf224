"""The reading behind the scaled FP64 solve: CG on S A S (S = diag(1/sqrt(d)),
d the diagonal of A) has the iterates of the diagonally preconditioned CG of A
under x~ = sqrt(d) x, r~ = r / sqrt(d), p~ = sqrt(d) p, with the same alpha,
beta and w.r, and the L1 norm of A's residual equal to sum |sqrt(d) r~|.

Checked here in plain numpy on matrices the oracle assembles (dense, small),
iteration by iteration, independently of the HIP path; and the diagonal PCG
written out here against the oracle's own PCG (same iterations, same x), so
that the comparison is tied to the oracle's conventions.
"""
import numpy as np
import pytest

import synth


def _dense(mesh, A):
    N = mesh.n_cells
    M = np.diag(np.asarray(A["diag_b"], dtype=np.float64))
    o, n = np.asarray(mesh.owner), np.asarray(mesh.neighbour)
    M[o, n] += A["upper"]
    M[n, o] += A["upper"]
    return M


def _pcg_diag(M, b, x0, iters):
    d = np.diag(M).copy()
    x = x0.copy()
    r = b - M @ x
    w = r / d
    wr = w @ r
    p = w.copy()
    out = []
    for _ in range(iters):
        q = M @ p
        alpha = wr / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        w = r / d
        wr_new = w @ r
        beta = wr_new / wr
        wr = wr_new
        p = w + beta * p
        out.append((alpha, beta, x.copy(), np.abs(r).sum()))
    return out


def _cg_scaled(M, b, x0, iters):
    sd = np.sqrt(np.diag(M))
    S = np.diag(1.0 / sd)
    At = S @ M @ S
    xt = sd * x0
    rt = (b - M @ x0) / sd
    p = rt.copy()
    rr = rt @ rt
    out = []
    for _ in range(iters):
        q = At @ p
        alpha = rr / (p @ q)
        xt = xt + alpha * p
        rt = rt - alpha * q
        rr_new = rt @ rt
        beta = rr_new / rr
        rr = rr_new
        p = rt + beta * p
        out.append((alpha, beta, xt / sd, np.abs(sd * rt).sum()))
    return out


CASES = [("graded_6x5x4", synth.box_mesh(6, 5, 4, z_ratio=4.0), 2e-3, 5e-3),
         ("paper_dt_5x4x3", synth.box_mesh(5, 4, 3), 1e-4, 0.2),
         ("skewed_5x4x4", synth.affine(synth.box_mesh(5, 4, 4, z_ratio=2.0), synth.SKEW), 2e-3, 5e-3)]


@pytest.mark.parametrize("name,mesh,DT,dt", CASES, ids=[c[0] for c in CASES])
def test_scaled_cg_has_the_diagonal_pcg_iterates(oracle, name, mesh, DT, dt):
    T0 = synth.initial_field(mesh.n_cells, 41)
    A = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    M = _dense(mesh, A)
    b = np.asarray(A["source_b"], dtype=np.float64)
    iters = 8
    ref, got = _pcg_diag(M, b, T0, iters), _cg_scaled(M, b, T0, iters)
    scale = np.abs(T0).max()
    for k, ((a0, b0, x0, n0), (a1, b1, x1, n1)) in enumerate(zip(ref, got)):
        assert abs(a1 - a0) <= 1e-11 * abs(a0), (name, k)
        assert abs(b1 - b0) <= 1e-9 * abs(b0) + 1e-300, (name, k)
        assert np.max(np.abs(x1 - x0)) <= 1e-12 * scale, (name, k)
        assert abs(n1 - n0) <= 1e-9 * n0 + 1e-12 * np.abs(b).sum(), (name, k)


@pytest.mark.parametrize("name,mesh,DT,dt", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_written_out_pcg_is_the_oracles(oracle, name, mesh, DT, dt):
    """The diagonal PCG above stopped after the oracle's iteration count gives
    the oracle's solution: the scaled form is compared with the method the
    oracle implements."""
    T0 = synth.initial_field(mesh.n_cells, 42)
    A = oracle.assemble(mesh, synth.fixed_x_bcs(), DT, dt, T0)
    x, st = oracle.pcg(mesh, A["diag_b"], A["upper"], A["source_b"], T0, tol=1e-9)
    n = st["n_iter"]
    assert n >= 2
    M = _dense(mesh, A)
    ref = _pcg_diag(M, np.asarray(A["source_b"], dtype=np.float64), T0, n)
    assert np.max(np.abs(ref[-1][2] - x)) <= 1e-11 * np.abs(x).max(), name
