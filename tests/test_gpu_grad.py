"""Gauss gradient on the GPU (lf_grad) against the oracle's sequential face
loop, on the same seeded inputs.

The kernel gathers each cell's faces in the order the face loop reaches the
cell and the library is built without multiply-add contraction, so the bar is
bit-exact equality of every gradient component, cell and boundary face.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam
from tests.helpers import tiny_face_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _strip_boundary(mesh):
    """The same cells and internal faces with no boundary patches (B = 0)."""
    return synth.BoxMesh(
        n_cells=mesh.n_cells, n_faces=mesh.n_faces, owner=mesh.owner, neighbour=mesh.neighbour,
        cell_volume=mesh.cell_volume, cell_centre=mesh.cell_centre, face_area=mesh.face_area,
        face_centre=mesh.face_centre, patch_names=(), patch_start=np.zeros(1, np.int32),
        bface_cell=np.zeros(0, np.int32), bface_area=np.zeros((0, 3)),
        bface_centre=np.zeros((0, 3)), shape=mesh.shape, ijk=mesh.ijk)


def _meshes():
    skew = lambda m: synth.affine(m, synth.SKEW)
    g = synth.box_mesh(9, 8, 7, z_ratio=4.0)                     # 504 cells: 2 workgroups, ragged
    yield "skew_graded_9x8x7", skew(g), True
    yield "skew_random_9x8x7", skew(synth.renumber(g, synth.random_permutation(g.n_cells, 3))), True
    big = synth.box_mesh(20, 17, 13, z_ratio=10.0)               # 4420 cells
    yield "graded_20x17x13", big, False
    yield "skew_random_20x17x13", skew(synth.renumber(big, synth.random_permutation(big.n_cells, 8))), True
    rb = synth.box_mesh(6, 5, 4)
    yield "redblack_6x5x4", synth.renumber(rb, synth.red_black_numbering(rb)[0]), False
    tiny = synth.box_mesh(3, 3, 2)
    yield "skew_random_3x3x2", skew(synth.renumber(tiny, synth.random_permutation(tiny.n_cells, 4))), True
    yield "line_9", synth.renumber(synth.box_mesh(9, 1, 1), synth.random_permutation(9, 6)), False
    yield "line_9_natural", synth.box_mesh(9, 1, 1, z_ratio=1.0), False
    yield "one_cell", skew(synth.box_mesh(1, 1, 1)), True
    yield "no_patches_5x4x3", _strip_boundary(skew(synth.box_mesh(5, 4, 3, z_ratio=2.0))), True
    # x and y faces past the limiter's angle (delta_f = 1/(0.05|d|)), band form and rows
    yield "steep_graded_9x8x7", synth.affine(g, synth.STEEP), True
    yield "steep_random_9x8x7", synth.affine(synth.renumber(g, synth.random_permutation(g.n_cells, 5)),
                                             synth.STEEP), True
    # a face whose interpolation weight takes the ROOTVSMALL fallback of 1/2
    yield "tiny_face_two_cells", tiny_face_cells(), True


MESHES = list(_meshes())


def _inputs(mesh, seed):
    T = synth.initial_field(mesh.n_cells, seed)
    Tb = synth.initial_field(mesh.n_bfaces, seed + 1)
    snb = 400.0 * (synth.uniform01(seed + 2, mesh.n_bfaces) - 0.5)
    return T, Tb, snb


def _gpu_grad(L, m, T, Tb, snb, with_boundary=True):
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    g, bg = m.grad(dev(T), dev(Tb), dev(snb), with_boundary=with_boundary)
    torch.cuda.synchronize()
    return g.cpu().numpy(), (bg.cpu().numpy() if bg is not None else None)


@pytest.mark.parametrize("name,mesh,skewed", MESHES, ids=[n for n, _, _ in MESHES])
def test_grad_bitwise(L, oracle, name, mesh, skewed):
    m = L.Mesh(mesh, gradient=True, non_orthogonal=skewed)
    T, Tb, snb = _inputs(mesh, 31)
    g, bg = _gpu_grad(L, m, T, Tb, snb)
    og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.array_equal(g, og), (name, float(np.max(np.abs(g - og))))
    assert np.array_equal(bg, obg), (name, float(np.max(np.abs(bg - obg))))
    # without the boundary gradient: the same cell gradient
    g2, none = _gpu_grad(L, m, T, Tb, snb, with_boundary=False)
    assert none is None and np.array_equal(g2, og)
    m.close()


def test_grad_repeated_calls_and_fields(L, oracle):
    """Two fields through one mesh, the second after the first: no state kept."""
    mesh = synth.affine(synth.box_mesh(11, 7, 5, z_ratio=3.0), synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    for seed in (41, 51):
        T, Tb, snb = _inputs(mesh, seed)
        g, bg = _gpu_grad(L, m, T, Tb, snb)
        og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
        assert np.array_equal(g, og) and np.array_equal(bg, obg), seed
    m.close()


def test_grad_linear_field_exact(L):
    """A property that holds at any size: the gradient of a linear field on a
    skewed graded box is its constant gradient (boundary values exact)."""
    mesh = synth.affine(synth.box_mesh(16, 12, 10, z_ratio=8.0), synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    gv = np.array([2.0, -1.5, 0.75])
    T = 10.0 + mesh.cell_centre @ gv
    Tb = 10.0 + mesh.bface_centre @ gv
    n = mesh.bface_area / np.sqrt((mesh.bface_area ** 2).sum(axis=1))[:, None]
    g, bg = _gpu_grad(L, m, T, Tb, n @ gv)
    assert np.max(np.abs(g - gv)) < 1e-10
    assert np.max(np.abs(bg - gv)) < 1e-10
    m.close()


def test_grad_errors(L):
    mesh = synth.affine(synth.box_mesh(3, 3, 3), synth.SKEW)
    # skewed faces need the flag
    with pytest.raises(L.LapfoamError, match="LF_EMESH"):
        L.Mesh(mesh, gradient=True)
    # a problem on a skewed mesh needs the face centres (its correction's gradient)
    bare = L.Mesh(mesh, non_orthogonal=True)
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        L.Problem(bare, synth.fixed_x_bcs(), 1.0, 0.1)
    bare.close()
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    # NULL boundary values with boundary faces present
    import torch
    T = torch.zeros(mesh.n_cells, dtype=torch.float64, device="cuda")
    g = torch.empty((mesh.n_cells, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        L.lf_grad(m.h, T.data_ptr(), 0, 0, g.data_ptr(), 0)
    m.close()
    # a mesh created without face centres holds no gradient geometry
    plain = L.Mesh(synth.box_mesh(3, 3, 3))
    Tb = torch.zeros(plain.n_bfaces, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        plain.grad(T, Tb, Tb)
    plain.close()


def test_grad_skewed_128(L, oracle):
    """128^3 skewed box (two cells per thread along z, 8192 workgroups):
    every output bit for bit."""
    mesh = synth.affine(synth.box_mesh(128, 128, 128, z_ratio=10.0), synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    assert m.n_bands == 3
    T, Tb, snb = _inputs(mesh, 71)
    g, bg = _gpu_grad(L, m, T, Tb, snb)
    m.close()
    og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.array_equal(g, og), float(np.max(np.abs(g - og)))
    assert np.array_equal(bg, obg), float(np.max(np.abs(bg - obg)))


def test_grad_full_size_skewed_256(L, oracle):
    """The 256^3 box graded in z (ratio 10), skewed: every output compared
    with the oracle, bit for bit, in the launch the benchmark times."""
    base = synth.build_config("graded_256").mesh
    mesh = synth.affine(base, synth.SKEW)
    del base
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    T, Tb, snb = _inputs(mesh, 61)
    g, bg = _gpu_grad(L, m, T, Tb, snb)
    m.close()
    og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.array_equal(g, og), float(np.max(np.abs(g - og)))
    assert np.array_equal(bg, obg), float(np.max(np.abs(bg - obg)))


def test_grad_full_size_permuted_192_skewed(L, oracle):
    """The row path at full size: the randomly numbered 192^3 box (kept by the
    library in Morton cell order), skewed; every output bit for bit."""
    mesh = synth.affine(synth.build_config("permuted_192").mesh, synth.SKEW)
    m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
    assert m.n_bands == 0 and m.cell_order()[0] == 1
    T, Tb, snb = _inputs(mesh, 81)
    g, bg = _gpu_grad(L, m, T, Tb, snb)
    m.close()
    og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.array_equal(g, og), float(np.max(np.abs(g - og)))
    assert np.array_equal(bg, obg), float(np.max(np.abs(bg - obg)))


PROBLEM_MESHES = [
    ("graded_9x8x7", synth.box_mesh(9, 8, 7, z_ratio=4.0), False),
    ("random_9x8x7", synth.renumber(synth.box_mesh(9, 8, 7, z_ratio=4.0),
                                    synth.random_permutation(504, 3)), False),
    ("skew_random_9x8x7", synth.affine(synth.renumber(synth.box_mesh(9, 8, 7, z_ratio=4.0),
                                                      synth.random_permutation(504, 3)), synth.SKEW), True),
    ("skew_graded_9x8x7", synth.affine(synth.box_mesh(9, 8, 7, z_ratio=4.0), synth.SKEW), True),
]


@pytest.mark.parametrize("name,mesh,skewed", PROBLEM_MESHES, ids=[n for n, _, _ in PROBLEM_MESHES])
def test_problem_grad_with_its_conditions(L, oracle, name, mesh, skewed):
    """The gradient of a problem's T with its own boundary conditions, bit for
    bit against the oracle's boundary values and gradient (mixed conditions)."""
    bcs = [(synth.FIXED_VALUE, 300.0), (synth.FIXED_VALUE, 500.0), (synth.ZERO_GRADIENT, 0.0),
           (synth.FIXED_VALUE, 410.0), (synth.ZERO_GRADIENT, 0.0), (synth.ZERO_GRADIENT, 0.0)]
    import torch
    m = L.Mesh(mesh, gradient=True, non_orthogonal=skewed)
    P = L.Problem(m, bcs, 1e-3, 5e-3)
    T = synth.initial_field(mesh.n_cells, 91)
    P.set_T(T)
    g, bg = P.grad()
    torch.cuda.synchronize()
    Tb, snb = oracle.boundary_values(mesh, bcs, T)
    og, obg = oracle.gauss_grad(mesh, T, Tb, snb)
    assert np.array_equal(g.cpu().numpy(), og), name
    assert np.array_equal(bg.cpu().numpy(), obg), name
    P.close()
    m.close()


def test_problem_grad_needs_face_centres(L):
    m = L.Mesh(synth.box_mesh(3, 3, 3))
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 5e-3)
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        P.grad()
    P.close()
    m.close()


def test_problem_grad_refused_while_stepping(L):
    """lf_problem_grad reads T: refused (LF_ESTATE) while an lf_step_begin run
    is in flight, allowed once it has finished."""
    import time
    mesh = synth.box_mesh(12, 10, 8)
    m = L.Mesh(mesh, gradient=True)
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 5e-3)
    P.set_T(synth.initial_field(mesh.n_cells, 3))
    P.step_begin(3)
    finished = False
    try:
        P.grad()
        refused = False
    except L.LapfoamError as e:
        refused = "LF_ESTATE" in str(e)
    t0 = time.time()
    while not finished and time.time() - t0 < 60:
        _, finished, _, _ = P.step_poll()
    assert finished
    # the run advances only through step_poll, so it was still in flight at the call
    assert refused
    g, _ = P.grad()
    assert g.shape == (mesh.n_cells, 3)
    P.close()
    m.close()
