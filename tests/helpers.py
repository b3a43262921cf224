"""Independent checkers used by the CPU pin tests.

Nothing here calls the oracle or the GPU library: these are second,
differently-structured derivations of what the method computes, used to pin
the oracle.
"""
import numpy as np


def stencil_system(mesh, bcs, DT, dt, T_old):
    """Dense A and b of one implicit-Euler step, built cell by cell on the box.

    Works from the (i, j, k) index of each cell and the node coordinates only
    (not from the face lists): for each of the six sides of a hexahedron, the
    two-point flux coefficient is DT * (side area) / (centre-to-centre distance
    along the axis); at a fixedValue wall the distance is centre-to-wall and the
    wall value goes to b; a zeroGradient wall adds nothing.  The time term adds
    V/dt to the diagonal and V/dt * T_old to b.
    """
    nx, ny, nz = mesh.shape
    xs, ys, zs = mesh.nodes
    nodes = (xs, ys, zs)
    cen = [0.5 * (a[:-1] + a[1:]) for a in nodes]
    wid = [np.diff(a) for a in nodes]
    N = mesh.n_cells
    A = np.zeros((N, N))
    b = np.zeros(N)
    # label of (i,j,k) in this (possibly renumbered) mesh
    lab = {tuple(mesh.ijk[c]): c for c in range(N)}
    dims = (nx, ny, nz)
    for c in range(N):
        ijk = mesh.ijk[c]
        V = wid[0][ijk[0]] * wid[1][ijk[1]] * wid[2][ijk[2]]
        A[c, c] += V / dt
        b[c] += V / dt * T_old[c]
        for axis in range(3):
            o1, o2 = [a for a in range(3) if a != axis]
            area = wid[o1][ijk[o1]] * wid[o2][ijk[o2]]
            for side in (-1, 1):
                q = ijk[axis] + side
                if 0 <= q < dims[axis]:
                    nb = list(ijk)
                    nb[axis] = q
                    dist = abs(cen[axis][q] - cen[axis][ijk[axis]])
                    a = DT * area / dist
                    A[c, c] += a
                    A[c, lab[tuple(nb)]] -= a
                else:
                    patch = 2 * axis + (1 if side > 0 else 0)
                    kind, value = bcs[patch]
                    if kind == 1:
                        wall = nodes[axis][dims[axis] if side > 0 else 0]
                        dist = abs(wall - cen[axis][ijk[axis]])
                        a = DT * area / dist
                        A[c, c] += a
                        b[c] += a * value
    return A, b


def ldu_to_dense(mesh, diag, upper):
    N = mesh.n_cells
    A = np.zeros((N, N))
    A[np.arange(N), np.arange(N)] = diag
    A[mesh.owner, mesh.neighbour] = upper
    A[mesh.neighbour, mesh.owner] = upper
    return A


def norm_factor(A, b, x0):
    """Normalisation factor of the residual, from its definition on a dense A."""
    row_sums = A.sum(axis=1)
    pA = row_sums * x0.mean()
    return np.sum(np.abs(A @ x0 - pA) + np.abs(b - pA)) + 1e-20


def line_mesh(n, z_ratio=1.0):
    import synth
    return synth.box_mesh(n, 1, 1, z_ratio=z_ratio)


def tiny_face_cells():
    """Two cells whose shared face reaches the interpolation weight's fallback.

    Cells at (0, 0, 0) and (1e-11, 1, 0) with volumes 1e-140; the internal face
    has S = (1e-140, 0, 0) and centre (2e-12, 0.5, 0), so its projected
    distances sum to 1e-151 (the weight is 1/2, against 0.8 from their ratio)
    and n.d = 1e-11 is far below 0.05|d| (the limiter binds).  Every area and
    volume is of order 1e-140, so the face's value weighs as much in the
    cells' gradients as on an ordinary mesh.  Six patches in the order of a
    box's (x walls first), the last four empty.
    """
    import synth
    s = 1e-140
    return synth.from_arrays(
        [[0.0, 0.0, 0.0], [1e-11, 1.0, 0.0]], [s, s],
        [(0, 1, (s, 0.0, 0.0), (2e-12, 0.5, 0.0))],
        [[(0, (-s, 0.0, 0.0), (-0.5, 0.0, 0.0))], [(1, (s, 0.0, 0.0), (0.5 + 1e-11, 1.0, 0.0))],
         [(0, (0.0, -s, 0.0), (0.0, -0.5, 0.0))], [(1, (0.0, s, 0.0), (1e-11, 1.5, 0.0))], [], []])
