"""Pins of the oracle's Gauss gradient against facts of the mathematics (no GPU).

A slip anywhere in the oracle's gradient fails one of these: swapped
interpolation weights (linear exactness on graded cells), a wrong sign or a
transposed owner/neighbour in the face loop (central differences), a dropped
boundary term or volume division (boundary cells, linear exactness), a wrong
sign or normalisation in the boundary correction (its normal component).
For the Laplacian's non-orthogonal correction: a wrong correction vector,
factor or sign fails the exact face flux of a linear field.
"""
import numpy as np
import pytest

import synth
from synth import FIXED_VALUE, ZERO_GRADIENT


def _skewed(shape, ratio, numbering="natural", seed=5):
    mesh = synth.affine(synth.box_mesh(*shape, z_ratio=ratio), synth.SKEW)
    if numbering == "random":
        mesh = synth.renumber(mesh, synth.random_permutation(mesh.n_cells, seed))
    return mesh


def _unit_normals(mesh):
    S = mesh.bface_area
    return S / np.sqrt((S * S).sum(axis=1))[:, None]


def test_weights_are_width_ratios_on_graded_skewed_box(oracle):
    """On a box graded in z and then skewed, the owner weight of the face
    between cells of widths h_P and h_N (along the face's axis) is
    h_N / (h_P + h_N): the map keeps ratios of lengths along a line."""
    nx, ny, nz = 3, 4, 6
    base = synth.box_mesh(nx, ny, nz, z_ratio=5.0)
    mesh = synth.affine(base, synth.SKEW)
    w = oracle.interp_weights(mesh)
    widths = [np.diff(x) for x in base.nodes]
    ijk = base.ijk
    want = np.empty(mesh.n_faces)
    for f in range(mesh.n_faces):
        P, N = mesh.owner[f], mesh.neighbour[f]
        axis = int(np.flatnonzero(ijk[N] != ijk[P])[0])
        hP, hN = widths[axis][ijk[P, axis]], widths[axis][ijk[N, axis]]
        want[f] = hN / (hP + hN)
    assert np.max(np.abs(w - want)) < 1e-13
    assert np.any(np.abs(want - 0.5) > 0.05)      # the grading makes them differ


@pytest.mark.parametrize("shape,ratio,numbering", [
    ((4, 3, 5), 1.0, "natural"), ((3, 4, 6), 6.0, "natural"), ((5, 4, 3), 3.0, "random"),
    ((1, 1, 1), 1.0, "natural"), ((6, 1, 1), 2.0, "random")])
def test_linear_field_gradient_exact_on_skewed_box(oracle, shape, ratio, numbering):
    """T = a + g.x on parallelepiped cells: linear interpolation is exact at
    each face centre and the face sum is the exact surface integral, so the
    Gauss gradient is g in every cell (boundary values given exactly).  The
    boundary gradient is g + n e when snGrad_b = g.n + e."""
    mesh = _skewed(shape, ratio, numbering)
    g = np.array([1.7, -2.3, 0.9])
    a = 3.25
    T = a + mesh.cell_centre @ g
    Tb = a + mesh.bface_centre @ g
    n = _unit_normals(mesh)
    e = synth.uniform01(21, mesh.n_bfaces) - 0.5
    snb = n @ g + e
    grad, bgrad = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.max(np.abs(grad - g)) < 1e-11
    assert np.max(np.abs(bgrad - (g + n * e[:, None]))) < 1e-11


@pytest.mark.parametrize("numbering", ["natural", "random"])
def test_central_differences_on_uniform_box(oracle, numbering):
    """On a uniform box the Gauss gradient of any field is the central
    difference (T_{i+1} - T_{i-1}) / (2h) inside; a boundary cell uses its face
    value: ((T_i + T_{i+1})/2 - T_b) / h at a low boundary."""
    nx, ny, nz = 5, 4, 3
    L = (1.0, 0.8, 0.45)
    mesh = synth.box_mesh(nx, ny, nz, lengths=L)
    if numbering == "random":
        mesh = synth.renumber(mesh, synth.random_permutation(mesh.n_cells, 9))
    T = synth.initial_field(mesh.n_cells, 4)
    Tb = 250.0 + 100.0 * synth.uniform01(8, mesh.n_bfaces)
    snb = np.zeros(mesh.n_bfaces)
    grad, _ = oracle.gauss_grad(mesh, T, Tb, snb)
    h = np.array([L[0] / nx, L[1] / ny, L[2] / nz])
    dims = (nx, ny, nz)
    cell_at = {tuple(ijk): c for c, ijk in enumerate(mesh.ijk)}
    bval = {}
    for p in range(6):
        axis, hi = p // 2, p % 2
        for b in range(mesh.patch_start[p], mesh.patch_start[p + 1]):
            bval[(int(mesh.bface_cell[b]), axis, hi)] = Tb[b]
    for c, ijk in enumerate(mesh.ijk):
        for axis in range(3):
            lo_ijk, hi_ijk = list(ijk), list(ijk)
            lo_ijk[axis] -= 1
            hi_ijk[axis] += 1
            lo = (T[cell_at[tuple(lo_ijk)]] + T[c]) / 2 if ijk[axis] > 0 else bval[(c, axis, 0)]
            up = (T[cell_at[tuple(hi_ijk)]] + T[c]) / 2 if ijk[axis] < dims[axis] - 1 \
                else bval[(c, axis, 1)]
            want = (up - lo) / h[axis]
            assert abs(grad[c, axis] - want) <= 1e-9 * max(1.0, abs(want)), (c, axis)


def test_divergence_identity(oracle):
    """Internal faces cancel in pairs: sum_c V_c g_c = sum_b S_b T_b for any
    cell field and boundary values (skewed, graded, randomly numbered)."""
    mesh = _skewed((5, 4, 6), 4.0, "random", seed=17)
    T = synth.initial_field(mesh.n_cells, 6)
    Tb = synth.initial_field(mesh.n_bfaces, 7)
    grad, _ = oracle.gauss_grad(mesh, T, Tb, np.zeros(mesh.n_bfaces))
    lhs = (mesh.cell_volume[:, None] * grad).sum(axis=0)
    rhs = (mesh.bface_area * Tb[:, None]).sum(axis=0)
    scale = np.abs(mesh.bface_area * Tb[:, None]).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale)


def test_boundary_correction_sets_normal_component(oracle):
    """n.g_b = snGrad_b and the tangential part is the face cell's gradient."""
    mesh = _skewed((4, 3, 3), 2.0)
    T = synth.initial_field(mesh.n_cells, 12)
    Tb = synth.initial_field(mesh.n_bfaces, 13)
    snb = 50.0 * (synth.uniform01(14, mesh.n_bfaces) - 0.5)
    grad, bgrad = oracle.gauss_grad(mesh, T, Tb, snb)
    n = _unit_normals(mesh)
    gP = grad[mesh.bface_cell]
    assert np.max(np.abs((n * bgrad).sum(axis=1) - snb)) < 1e-9
    tang_b = bgrad - n * (n * bgrad).sum(axis=1)[:, None]
    tang_P = gP - n * (n * gP).sum(axis=1)[:, None]
    assert np.max(np.abs(tang_b - tang_P)) < 1e-9


def test_boundary_values_of_the_conditions(oracle):
    """fixedValue: T_b = value, snGrad = (value - T_P) / (h/2) on a uniform
    box; zeroGradient: T_b = T_P, snGrad = 0."""
    nx, ny, nz = 4, 3, 2
    mesh = synth.box_mesh(nx, ny, nz)
    bcs = [(FIXED_VALUE, 300.0), (FIXED_VALUE, 500.0), (ZERO_GRADIENT, 0.0),
           (FIXED_VALUE, 410.0), (ZERO_GRADIENT, 0.0), (ZERO_GRADIENT, 0.0)]
    T = synth.initial_field(mesh.n_cells, 2)
    Tb, snb = oracle.boundary_values(mesh, bcs, T)
    half = (0.5 / nx, 0.5 / ny, 0.5 / nz)
    for p, (kind, val) in enumerate(bcs):
        for b in range(mesh.patch_start[p], mesh.patch_start[p + 1]):
            Tc = T[mesh.bface_cell[b]]
            if kind == FIXED_VALUE:
                assert Tb[b] == val
                assert abs(snb[b] - (val - Tc) / half[p // 2]) < 1e-9 * abs(val)
            else:
                assert Tb[b] == Tc and snb[b] == 0.0


# --------------------------------------------------------------------------
# the Laplacian's explicit non-orthogonal correction
# --------------------------------------------------------------------------
def _laplacian_of(mesh, A, lap_src, T):
    """Per cell: sum over its internal faces of lapU_f (T_other - T_c) minus
    the explicit source (the discrete laplacian the corrected scheme applies;
    lapU_f = -upper_f)."""
    lapU = -A["upper"]
    out = np.zeros(mesh.n_cells)
    np.add.at(out, mesh.owner, lapU * (T[mesh.neighbour] - T[mesh.owner]))
    np.add.at(out, mesh.neighbour, lapU * (T[mesh.owner] - T[mesh.neighbour]))
    scale = np.zeros(mesh.n_cells)
    np.add.at(scale, mesh.owner, np.abs(lapU * (T[mesh.neighbour] - T[mesh.owner])))
    np.add.at(scale, mesh.neighbour, np.abs(lapU * (T[mesh.owner] - T[mesh.neighbour])))
    return out - lap_src, scale


@pytest.mark.parametrize("shape", [(2, 1, 1), (1, 2, 1), (1, 1, 2)])
def test_corrected_face_flux_is_exact_for_linear_field(oracle, shape):
    """Two skewed cells, one face: the implicit flux DT|S| delta (T_N - T_P)
    plus the correction DT|S| k.g (n = delta d + k) is the exact flux DT S.g
    of a linear field, which the implicit part alone misses on a skewed face.
    With one face, lap_src of the owner is minus that face's correction."""
    mesh = synth.affine(synth.box_mesh(*shape, lengths=(0.5, 0.7, 0.9)), synth.SKEW)
    assert mesh.n_faces == 1
    g = np.array([1.7, -2.3, 0.9])
    T = 3.25 + mesh.cell_centre @ g
    grad, _ = oracle.gauss_grad(mesh, T, 3.25 + mesh.bface_centre @ g, np.zeros(mesh.n_bfaces))
    DT = 0.7
    lap_src = oracle.nonorth_source(mesh, DT, grad)
    A = oracle.assemble(mesh, synth.all_zero_gradient(), DT, 0.1, T, lap_src=lap_src)
    implicit = -A["upper"][0] * (T[1] - T[0])
    exact = DT * (mesh.face_area[0] @ g)
    assert abs(implicit - lap_src[0] - exact) < 1e-12 * abs(exact)
    assert abs(lap_src[0] + lap_src[1]) < 1e-15 * abs(exact)
    assert abs(implicit - exact) > 1e-2 * abs(exact)


@pytest.mark.parametrize("numbering", ["natural", "random"])
def test_corrected_laplacian_of_linear_field_vanishes(oracle, numbering):
    """With the correction the face flux is DT S_f.g for a linear field, so
    every cell without boundary faces has zero net flux."""
    mesh = _skewed((6, 5, 7), 3.0, numbering)
    g = np.array([1.7, -2.3, 0.9])
    T = 3.25 + mesh.cell_centre @ g
    grad, _ = oracle.gauss_grad(mesh, T, 3.25 + mesh.bface_centre @ g, np.zeros(mesh.n_bfaces))
    DT = 0.7
    lap_src = oracle.nonorth_source(mesh, DT, grad)
    A = oracle.assemble(mesh, synth.all_zero_gradient(), DT, 0.1, T, lap_src=lap_src)
    inner = np.ones(mesh.n_cells, bool)
    inner[mesh.bface_cell] = False
    assert inner.sum() > 20
    L, scale = _laplacian_of(mesh, A, lap_src, T)
    assert np.max(np.abs(L[inner]) / scale[inner]) < 1e-12


def test_correction_vanishes_on_orthogonal_box(oracle):
    """k_f = n_f - delta_f d_f is exactly zero on an axis-aligned box."""
    mesh = synth.box_mesh(5, 4, 6, z_ratio=4.0)
    T = synth.initial_field(mesh.n_cells, 3)
    lap_src = oracle.step_source(mesh, synth.fixed_x_bcs(), 0.5, T)
    assert np.all(lap_src == 0.0)


def test_correction_enters_the_source(oracle):
    """TEqn's source is the ddt source minus the laplacian's explicit source."""
    mesh = _skewed((4, 3, 5), 2.0)
    T = synth.initial_field(mesh.n_cells, 4)
    bcs = synth.fixed_x_bcs()
    lap_src = oracle.step_source(mesh, bcs, 0.4, T)
    A0 = oracle.assemble(mesh, bcs, 0.4, 0.05, T)
    A1 = oracle.assemble(mesh, bcs, 0.4, 0.05, T, lap_src=lap_src)
    assert np.array_equal(A1["source"], A0["source"] - lap_src)
    assert np.array_equal(A1["diag"], A0["diag"]) and np.array_equal(A1["upper"], A0["upper"])
    assert np.max(np.abs(lap_src)) > 0.0


def test_corrected_steps_conserve_heat(oracle):
    """All walls zeroGradient: internal faces cancel in the sum of the
    explicit source, so sum V T is kept to the solver tolerance."""
    mesh = _skewed((5, 4, 4), 2.0, "random")
    T0 = synth.initial_field(mesh.n_cells, 8)
    T, stats, _ = oracle.run_nonorth(mesh, synth.all_zero_gradient(), 0.05, 0.01, 3, T0,
                                     tol=1e-13)
    h0, h1 = (mesh.cell_volume * T0).sum(), (mesh.cell_volume * T).sum()
    assert abs(h1 - h0) <= 1e-10 * h0
    assert all(s["converged"] for s in stats)


def test_corrector_passes_converge_to_the_corrected_fixed_point(oracle):
    """More passes of the corrector loop solve the step's implicit-in-the-
    correction system ever more closely: the change from pass n to n+1 shrinks,
    and with no correction (an orthogonal box) extra passes change nothing."""
    mesh = _skewed((6, 5, 4), 3.0)
    T0 = synth.initial_field(mesh.n_cells, 9)
    bcs, DT, dt = synth.fixed_x_bcs(), 0.05, 0.02
    Ts = [oracle.run_nonorth(mesh, bcs, DT, dt, 1, T0, tol=1e-14, n_corr=k)[0] for k in range(4)]
    d = [np.max(np.abs(Ts[k + 1] - Ts[k])) for k in range(3)]
    assert d[0] > 0.0 and d[1] < 0.5 * d[0] and d[2] < 0.5 * d[1], d
    box = synth.box_mesh(5, 4, 3)
    T1 = oracle.run_nonorth(box, bcs, DT, dt, 1, T0[:box.n_cells], tol=1e-14)[0]
    T3 = oracle.run_nonorth(box, bcs, DT, dt, 1, T0[:box.n_cells], tol=1e-14, n_corr=2)[0]
    assert np.max(np.abs(T3 - T1)) <= 1e-9 * np.max(np.abs(T1))
