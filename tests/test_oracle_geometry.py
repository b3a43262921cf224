"""Pins of the oracle's face factors on faces that are not orthogonal to the
line joining their cell centres (no GPU).

The flux pins of the corrected scheme hold for any choice of delta (the
implicit part delta d.g plus the correction (n - delta d).g is n.g whatever
delta is), so the factors themselves are pinned here by hand-computed values:
  - delta_f = 1/(n.d) on a skewed face, not 1/|d| (the orthogonal part of the
    over-relaxed decomposition: its correction vector n - delta d is
    perpendicular to n);
  - delta_f = 1/(0.05|d|) where n.d < 0.05|d| (the limiter);
  - delta_b = 1/(n.(C_b - C_P)) on a skewed boundary face, not 1/|C_b - C_P|;
  - the interpolation weight 1/2 when the two projected distances sum to no
    more than ROOTVSMALL (Section 5.2, the weights listing; 1e-150, the
    double-precision value).

Each pin is a plain function of the oracle module so that
test_oracle_mutants.py can run the same pins against oracles with planted
mistakes.
"""
import numpy as np

import synth

DT, DTIME = 0.01, 0.1


def _two_cells(centre_n, patches=True):
    """Cell 0 at the origin, cell 1 at centre_n, unit volumes, one internal face
    with S = (2, 0, 0); with patches: a fixedValue patch holding one skewed
    boundary face of cell 0 (S_b = (-3, 0, 0), C_b - C_P = (-0.5, 0.4, -0.2)) and
    a zeroGradient patch holding one face of cell 1."""
    cn = np.asarray(centre_n, dtype=np.float64)
    pts = [[(0, (-3.0, 0.0, 0.0), (-0.5, 0.4, -0.2))],
           [(1, (3.0, 0.0, 0.0), tuple(cn + (0.5, 0.0, 0.0)))]] if patches else []
    return synth.from_arrays([[0.0, 0.0, 0.0], cn], [1.0, 1.0],
                             [(0, 1, (2.0, 0.0, 0.0), tuple(0.5 * cn))], pts)


def pin_two_cell_skewed_coefficients(O):
    """d = (1, 0.5, 0.25), n = (1, 0, 0): n.d = 1 is above 0.05|d| = 0.057, so
    delta_f = 1 and upper = -DT |S| delta_f = -0.02 (1/|d| would give -0.01746).
    The boundary face: n_b = (-1, 0, 0), n_b.(C_b - C_P) = 0.5, delta_b = 2,
    internal coefficient DT |S_b| delta_b = 0.06 (1/|C_b - C_P| = 1.49 would
    give 0.0447), boundary coefficient 0.06 * 300 = 18."""
    m = _two_cells((1.0, 0.5, 0.25))
    A = O.assemble(m, [(synth.FIXED_VALUE, 300.0), (synth.ZERO_GRADIENT, 0.0)], DT, DTIME,
                   np.array([280.0, 320.0]))
    assert abs(A["upper"][0] - (-0.02)) <= 1e-16, A["upper"]
    assert abs(A["int_coeff"][0] - 0.06) <= 1e-16, A["int_coeff"]
    assert abs(A["bou_coeff"][0] - 18.0) <= 1e-13, A["bou_coeff"]
    # V/dt + 0.02 (+ 0.06 on the fixedValue side); sources V/dt T_old (+ 18)
    assert np.allclose(A["diag_b"], [10.08, 10.02], rtol=0, atol=1e-13), A["diag_b"]
    assert np.allclose(A["source_b"], [2818.0, 3200.0], rtol=0, atol=1e-11), A["source_b"]


def pin_two_cell_limiter(O):
    """d = (1, 30, 0): n.d = 1 is below 0.05|d| = 0.05 sqrt(901) = 1.5008, so the
    limiter sets delta_f = 1/1.5008 and upper = -0.02/1.5008 = -0.013326."""
    m = _two_cells((1.0, 30.0, 0.0), patches=False)
    A = O.assemble(m, [], DT, DTIME, np.array([280.0, 320.0]))
    want = -DT * 2.0 / (0.05 * np.sqrt(901.0))
    assert abs(A["upper"][0] - want) <= 1e-16, (A["upper"], want)


def pin_steep_box_factors(O):
    """A uniform box sheared by synth.STEEP (x += 25 y).  Area vectors map by
    A^-T: an x face (a, 0, 0) becomes (a, -25a, 0), a y face stays (0, a, 0);
    centre offsets map by A: (h, 0, 0) stays, (0, h, 0) becomes (25h, h, 0).
    So the cosine between n and d is 1/sqrt(626) = 0.03997 < 0.05 on x and y
    faces, where the limiter binds:
      x faces: |d| = hx, delta = 1/(0.05 hx) = 20/hx;
      y faces: |d| = sqrt(626) hy, delta = 20/(sqrt(626) hy);
      z faces: orthogonal, delta = 1/hz.
    Boundary faces (no limiter: n.(C_b - C_P) is the distance itself):
      x walls: n.(C_b - C_P) = (hx/2)/sqrt(626), delta_b = 2 sqrt(626)/hx;
      y walls: n.(C_b - C_P) = hy/2, delta_b = 2/hy; z walls 2/hz."""
    nx, ny, nz = 4, 3, 5
    L = (1.0, 0.6, 0.5)
    base = synth.box_mesh(nx, ny, nz, lengths=L)
    mesh = synth.affine(base, synth.STEEP)
    h = np.array([L[0] / nx, L[1] / ny, L[2] / nz])
    r = np.sqrt(626.0)
    want_f = {0: 20.0 / h[0], 1: 20.0 / (r * h[1]), 2: 1.0 / h[2]}
    want_b = {0: 2.0 * r / h[0], 1: 2.0 / h[1], 2: 2.0 / h[2]}
    _, delta = O.face_geometry(mesh)
    ijk = base.ijk
    seen = set()
    for f in range(mesh.n_faces):
        axis = int(np.flatnonzero(ijk[mesh.neighbour[f]] != ijk[mesh.owner[f]])[0])
        seen.add(axis)
        assert abs(delta[f] - want_f[axis]) <= 1e-12 * want_f[axis], (f, axis, delta[f], want_f[axis])
    assert seen == {0, 1, 2}
    _, bdelta = O.bface_geometry(mesh)
    for p in range(6):
        axis = p // 2
        for b in range(mesh.patch_start[p], mesh.patch_start[p + 1]):
            assert abs(bdelta[b] - want_b[axis]) <= 1e-12 * want_b[axis], (p, b, bdelta[b])


def pin_weight_fallback(O):
    """Cells at (0,0,0) and (1e-11, 1, 0), face centre (2e-12, 0.5, 0), S = (s, 0, 0):
    SfdOwn = 2e-12 s and SfdNei = 8e-12 s, whose ratio gives the owner weight
    0.8 -- while their sum 1e-11 s is above 1e-150; at or below it the weight
    is 1/2."""
    def weight(s):
        m = synth.from_arrays([[0.0, 0.0, 0.0], [1e-11, 1.0, 0.0]], [1.0, 1.0],
                              [(0, 1, (s, 0.0, 0.0), (2e-12, 0.5, 0.0))], [])
        return float(O.interp_weights(m)[0])
    assert weight(1e-139) == 0.5          # sum rounds to just below 1e-150
    assert weight(1e-141) == 0.5          # sum 1e-152
    assert abs(weight(1.000001e-139) - 0.8) <= 1e-15    # sum just above 1e-150
    assert abs(weight(1e-120) - 0.8) <= 1e-15
    assert abs(weight(1.0) - 0.8) <= 1e-15


PINS = [pin_two_cell_skewed_coefficients, pin_two_cell_limiter, pin_steep_box_factors,
        pin_weight_fallback]


def test_two_cell_skewed_coefficients(oracle):
    pin_two_cell_skewed_coefficients(oracle)


def test_two_cell_limiter(oracle):
    pin_two_cell_limiter(oracle)


def test_steep_box_factors(oracle):
    pin_steep_box_factors(oracle)


def test_weight_fallback(oracle):
    pin_weight_fallback(oracle)
