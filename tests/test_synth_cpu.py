"""The skewed (affine) meshes the gradient and correction tests run on are
valid finite-volume meshes (no GPU): every cell closed, volumes and centres
mapped consistently, faces really non-orthogonal."""
import numpy as np

import synth


def _cell_area_sums(mesh):
    tot = np.zeros((mesh.n_cells, 3))
    np.add.at(tot, mesh.owner, mesh.face_area)
    np.add.at(tot, mesh.neighbour, -mesh.face_area)
    np.add.at(tot, mesh.bface_cell, mesh.bface_area)
    return tot


def test_affine_mesh_cells_are_closed_and_consistent():
    base = synth.box_mesh(5, 4, 3, z_ratio=3.0)
    A = np.asarray(synth.SKEW)
    mesh = synth.affine(base, A)
    scale = np.abs(mesh.face_area).max()
    assert np.abs(_cell_area_sums(mesh)).max() < 1e-14 * scale * 10
    assert np.allclose(mesh.cell_volume, np.linalg.det(A) * base.cell_volume, rtol=1e-14)
    assert np.isclose(mesh.cell_volume.sum(), np.linalg.det(A), rtol=1e-13)
    assert np.allclose(mesh.cell_centre, base.cell_centre @ A.T, rtol=0, atol=1e-15)
    # divergence theorem per cell for the position field: sum_f S_f . x_f = 3 V
    xs = np.zeros(mesh.n_cells)
    np.add.at(xs, mesh.owner, (mesh.face_area * mesh.face_centre).sum(axis=1))
    np.add.at(xs, mesh.neighbour, -(mesh.face_area * mesh.face_centre).sum(axis=1))
    np.add.at(xs, mesh.bface_cell, (mesh.bface_area * mesh.bface_centre).sum(axis=1))
    assert np.allclose(xs, 3.0 * mesh.cell_volume, rtol=1e-12)


def test_affine_faces_are_non_orthogonal_but_oriented():
    mesh = synth.affine(synth.box_mesh(4, 4, 4), synth.SKEW)
    d = mesh.cell_centre[mesh.neighbour] - mesh.cell_centre[mesh.owner]
    S = mesh.face_area
    cos = (S * d).sum(axis=1) / (np.linalg.norm(S, axis=1) * np.linalg.norm(d, axis=1))
    assert np.all(cos > 0.5)                 # owner -> neighbour orientation kept
    assert np.all(cos < 0.999)               # every face skewed
    bout = ((mesh.bface_centre - mesh.cell_centre[mesh.bface_cell]) * mesh.bface_area).sum(axis=1)
    assert np.all(bout > 0.0)                # boundary faces point outward
