"""lf_grad_noalloc (the gradient for callers that cannot allocate device
memory) against lf_grad through the C ABI: bitwise the same gradient on two
calls in a row, the second on a smaller mesh (the scratch array keeps the
first call's contents), on meshes kept in Morton order (the scratch is used)
and with band form (no scratch); the size limit of the scratch is refused."""
import numpy as np
import pytest

import synth
from tests.gpu_common import lapfoam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _inputs(mesh, seed):
    T = synth.initial_field(mesh.n_cells, seed)
    Tb = synth.initial_field(mesh.n_bfaces, seed + 1)
    snb = 400.0 * (synth.uniform01(seed + 2, mesh.n_bfaces) - 0.5)
    return T, Tb, snb


def _both(L, m, mesh, seed):
    """(lf_grad, lf_grad_noalloc) gradients and boundary gradients, host arrays."""
    import torch
    N, B = mesh.n_cells, mesh.n_bfaces
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    T, Tb, snb = (dev(a) for a in _inputs(mesh, seed))
    out = []
    for fn in (L.lf_grad, L.lf_grad_noalloc):
        g = torch.full((N, 3), float("nan"), dtype=torch.float64, device="cuda")
        bg = torch.full((max(B, 1), 3), float("nan"), dtype=torch.float64, device="cuda")
        fn(m.h, T.data_ptr(), Tb.data_ptr(), snb.data_ptr(), g.data_ptr(), bg.data_ptr())
        torch.cuda.synchronize()
        out.append((g.cpu().numpy(), bg[:B].cpu().numpy()))
    return out


def _skewed_random(nx, ny, nz, seed):
    g = synth.box_mesh(nx, ny, nz, z_ratio=4.0)
    return synth.affine(synth.renumber(g, synth.random_permutation(g.n_cells, seed)), synth.SKEW)


@pytest.mark.parametrize("kind", ["morton", "bands"])
def test_noalloc_equals_grad_twice_second_smaller(L, oracle, kind):
    if kind == "morton":
        meshes = [_skewed_random(24, 19, 15, 3), _skewed_random(9, 8, 7, 5)]
    else:
        meshes = [synth.affine(synth.box_mesh(24, 19, 15, z_ratio=4.0), synth.SKEW),
                  synth.affine(synth.box_mesh(9, 8, 7, z_ratio=2.0), synth.SKEW)]
    assert meshes[1].n_cells < meshes[0].n_cells
    for i, mesh in enumerate(meshes):
        m = L.Mesh(mesh, gradient=True, non_orthogonal=True)
        assert m.cell_order()[0] == (kind == "morton"), kind
        (g, bg), (gn, bgn) = _both(L, m, mesh, 31 + i)
        assert np.array_equal(g, gn), (kind, i)
        assert np.array_equal(bg, bgn), (kind, i)
        og, obg = oracle.gauss_grad(mesh, *_inputs(mesh, 31 + i))
        assert np.array_equal(gn, og) and np.array_equal(bgn, obg), (kind, i)
        m.close()


def test_noalloc_refuses_a_mesh_beyond_its_scratch(L):
    """A mesh in Morton order with more cells than the scratch holds (2^23)."""
    import torch
    g = synth.box_mesh(256, 256, 129)             # 8,454,144 cells
    mesh = synth.renumber(g, synth.random_permutation(g.n_cells, 7))
    assert mesh.n_cells > 1 << 23
    m = L.Mesh(mesh, gradient=True)
    assert m.cell_order()[0]
    N, B = mesh.n_cells, mesh.n_bfaces
    T = torch.zeros(N, dtype=torch.float64, device="cuda")
    Tb = torch.zeros(B, dtype=torch.float64, device="cuda")
    gr = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LapfoamError, match="scratch holds at most 8388608"):
        L.lf_grad_noalloc(m.h, T.data_ptr(), Tb.data_ptr(), 0, gr.data_ptr(), 0)
    # the allocating entry point still takes it
    L.lf_grad(m.h, T.data_ptr(), Tb.data_ptr(), 0, gr.data_ptr(), 0)
    torch.cuda.synchronize()
    assert float(gr.abs().max()) == 0.0
    m.close()


def test_noalloc_argument_checks(L):
    mesh = synth.box_mesh(4, 3, 2)
    m = L.Mesh(mesh)                  # no gradient geometry
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        L.lf_grad_noalloc(m.h, 0, 0, 0, 0, 0)
    m.close()
