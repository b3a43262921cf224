"""Hexahedral box meshes in OpenFOAM face addressing.

A mesh is described the way the paper states the problem (Section 4): cells,
internal faces with an owner and a neighbour label (the face area vector points
from owner to neighbour), and boundary faces grouped into patches, each
boundary face having only an owner ("face cell").

Internal faces are in upper-triangular order: owner < neighbour, and faces
sorted by (owner, neighbour).  Cell label c = i + nx*(j + ny*k).

Only geometry and numbering are generated here; every coefficient of the
discretisation is left to the code under test and to the oracle.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

from .rng import splitmix64, uniform01

PATCH_NAMES = ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax")


@dataclass
class BoxMesh:
    n_cells: int
    n_faces: int                      # internal faces
    owner: np.ndarray                 # int32[F]
    neighbour: np.ndarray             # int32[F]
    cell_volume: np.ndarray           # f64[N]
    cell_centre: np.ndarray           # f64[N,3]
    face_area: np.ndarray             # f64[F,3]  S_f, owner -> neighbour
    face_centre: np.ndarray           # f64[F,3]
    patch_names: Tuple[str, ...]
    patch_start: np.ndarray           # int32[P+1] into the boundary-face arrays
    bface_cell: np.ndarray            # int32[B]
    bface_area: np.ndarray            # f64[B,3]  outward
    bface_centre: np.ndarray          # f64[B,3]
    shape: Tuple[int, int, int] = (0, 0, 0)
    ijk: np.ndarray = field(default=None)       # int32[N,3] (i,j,k) of each cell label
    nodes: Tuple[np.ndarray, ...] = field(default=None)

    @property
    def n_patches(self) -> int:
        return len(self.patch_names)

    @property
    def n_bfaces(self) -> int:
        return int(self.bface_cell.shape[0])


def graded_nodes(n: int, ratio: float = 1.0, length: float = 1.0) -> np.ndarray:
    """Node coordinates of n cells on [0, length].

    ratio is the blockMesh expansion ratio (last cell width / first cell
    width); widths grow geometrically with r = ratio**(1/(n-1)).  The last node
    is set to `length` exactly.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    if ratio == 1.0 or n == 1:
        x = np.arange(n + 1, dtype=np.float64) * (length / n)
    else:
        r = ratio ** (1.0 / (n - 1))
        w0 = length * (r - 1.0) / (r ** n - 1.0)
        widths = w0 * r ** np.arange(n, dtype=np.float64)
        x = np.concatenate(([0.0], np.cumsum(widths)))
    x[0] = 0.0
    x[-1] = length
    return x


def box_mesh(nx: int, ny: int, nz: int, z_ratio: float = 1.0,
             lengths=(1.0, 1.0, 1.0)) -> BoxMesh:
    """Box [0,Lx]x[0,Ly]x[0,Lz] with nx*ny*nz hexahedra, graded in z."""
    xs = graded_nodes(nx, 1.0, lengths[0])
    ys = graded_nodes(ny, 1.0, lengths[1])
    zs = graded_nodes(nz, z_ratio, lengths[2])
    dx, dy, dz = np.diff(xs), np.diff(ys), np.diff(zs)
    xc, yc, zc = 0.5 * (xs[:-1] + xs[1:]), 0.5 * (ys[:-1] + ys[1:]), 0.5 * (zs[:-1] + zs[1:])
    N = nx * ny * nz
    shp = (nz, ny, nx)                      # C order: label = i + nx*(j + ny*k)
    X = (slice(None), None, None)
    Y = (None, slice(None), None)
    Z = (None, None, slice(None))
    lab = np.arange(N, dtype=np.int32).reshape(shp)
    vol = (dz[X] * dy[Y] * dx[Z]).reshape(-1)
    centre = np.empty(shp + (3,))
    centre[..., 0] = xc[Z]
    centre[..., 1] = yc[Y]
    centre[..., 2] = zc[X]

    # internal faces: per owner cell the +x, +y, +z neighbours, in that
    # (ascending-label) order, so (cell, direction) order is upper-triangular.
    # Each direction's faces are generated in owner order and scattered to
    # their position start[owner] + (number of earlier directions present).
    vx = np.zeros(shp, dtype=np.int64)
    vy = np.zeros(shp, dtype=np.int64)
    vz = np.zeros(shp, dtype=np.int64)
    vx[:, :, :-1] = 1
    vy[:, :-1, :] = 1
    vz[:-1, :, :] = 1
    cnt = (vx + vy + vz).reshape(-1)
    F = int(cnt.sum())
    start = (np.cumsum(cnt) - cnt).reshape(shp)
    sel = ((slice(None), slice(None), slice(0, nx - 1)),
           (slice(None), slice(0, ny - 1), slice(None)),
           (slice(0, nz - 1), slice(None), slice(None)))
    pos = [start[sel[0]].reshape(-1), (start + vx)[sel[1]].reshape(-1),
           (start + vx + vy)[sel[2]].reshape(-1)]
    del vx, vy, vz, start
    owner = np.empty(F, dtype=np.int32)
    neighbour = np.empty(F, dtype=np.int32)
    farea = np.zeros((F, 3))
    fcen = np.empty((F, 3))
    steps = (1, nx, nx * ny)
    area_full = (lambda: dz[X] * dy[Y] * np.ones(nx)[Z],
                 lambda: dz[X] * np.ones(ny)[Y] * dx[Z],
                 lambda: np.ones(nz)[X] * dy[Y] * dx[Z])
    node_hi = (xs[1:][Z], ys[1:][Y], zs[1:][X])
    for d in range(3):
        s, p = sel[d], pos[d]
        o = lab[s].reshape(-1)
        owner[p] = o
        neighbour[p] = o + steps[d]
        farea[p, d] = np.broadcast_to(area_full[d](), shp)[s].reshape(-1)
        for comp in range(3):
            src_ = node_hi[comp] if comp == d else (xc[Z], yc[Y], zc[X])[comp]
            fcen[p, comp] = np.broadcast_to(src_, shp)[s].reshape(-1)

    # boundary patches xmin, xmax, ymin, ymax, zmin, zmax; faces in cell order
    bcell, barea, bcen, pstart = [], [], [], [0]
    for p in range(6):
        axis, hi = p // 2, p % 2
        sl = [slice(None)] * 3
        sl[2 - axis] = -1 if hi else 0
        sl = tuple(sl)
        cells = lab[sl].reshape(-1)
        sgn = 1.0 if hi else -1.0
        a = np.zeros((cells.size, 3))
        full = np.zeros(shp)
        if axis == 0:
            full[...] = dz[X] * dy[Y] * np.ones(nx)[Z]
        elif axis == 1:
            full[...] = dz[X] * np.ones(ny)[Y] * dx[Z]
        else:
            full[...] = np.ones(nz)[X] * dy[Y] * dx[Z]
        a[:, axis] = sgn * full[sl].reshape(-1)
        f = centre[sl].reshape(-1, 3).copy()
        f[:, axis] = ((xs, ys, zs)[axis])[-1 if hi else 0]
        bcell.append(cells)
        barea.append(a)
        bcen.append(f)
        pstart.append(pstart[-1] + cells.size)

    ijk = np.empty(shp + (3,), dtype=np.int32)
    ijk[..., 0] = np.arange(nx, dtype=np.int32)[Z]
    ijk[..., 1] = np.arange(ny, dtype=np.int32)[Y]
    ijk[..., 2] = np.arange(nz, dtype=np.int32)[X]
    return BoxMesh(
        n_cells=N, n_faces=int(owner.size), owner=np.ascontiguousarray(owner),
        neighbour=np.ascontiguousarray(neighbour),
        cell_volume=vol, cell_centre=centre.reshape(-1, 3), face_area=farea, face_centre=fcen,
        patch_names=PATCH_NAMES, patch_start=np.asarray(pstart, dtype=np.int32),
        bface_cell=np.concatenate(bcell).astype(np.int32),
        bface_area=np.concatenate(barea), bface_centre=np.concatenate(bcen),
        shape=(nx, ny, nz), ijk=ijk.reshape(-1, 3), nodes=(xs, ys, zs))


def renumber(mesh: BoxMesh, new_of_old: np.ndarray) -> BoxMesh:
    """Relabel cells (cell c -> new_of_old[c]) and restore upper-triangular order.

    Each internal face takes owner = min and neighbour = max of its two new
    labels; when that swaps the two cells the face area vector is reversed so
    it still points owner -> neighbour.  Faces are then sorted by
    (owner, neighbour).  Boundary faces keep their order; only their face cell
    is relabelled.
    """
    new_of_old = np.asarray(new_of_old, dtype=np.int64)
    N = mesh.n_cells
    if new_of_old.shape != (N,) or not np.array_equal(np.sort(new_of_old), np.arange(N)):
        raise ValueError("new_of_old must be a permutation of the cell labels")
    old_of_new = np.empty(N, dtype=np.int64)
    old_of_new[new_of_old] = np.arange(N)
    a = new_of_old[mesh.owner]
    b = new_of_old[mesh.neighbour]
    swap = a > b
    own = np.where(swap, b, a)
    nei = np.where(swap, a, b)
    area = mesh.face_area.copy()
    area[swap] *= -1.0
    order = np.lexsort((nei, own))
    return BoxMesh(
        n_cells=N, n_faces=mesh.n_faces,
        owner=own[order].astype(np.int32), neighbour=nei[order].astype(np.int32),
        cell_volume=mesh.cell_volume[old_of_new], cell_centre=mesh.cell_centre[old_of_new],
        face_area=area[order], face_centre=mesh.face_centre[order],
        patch_names=mesh.patch_names, patch_start=mesh.patch_start.copy(),
        bface_cell=new_of_old[mesh.bface_cell].astype(np.int32),
        bface_area=mesh.bface_area.copy(), bface_centre=mesh.bface_centre.copy(),
        shape=mesh.shape, ijk=mesh.ijk[old_of_new] if mesh.ijk is not None else None,
        nodes=mesh.nodes)


def affine(mesh: BoxMesh, A) -> BoxMesh:
    """The mesh mapped by the linear map x -> A x (det A > 0): a box becomes a
    skewed box of parallelepiped cells whose faces are not orthogonal to the
    lines joining cell centres.  Centres map by A, area vectors by
    det(A) A^-T, volumes by det(A); numbering and patches are unchanged."""
    A = np.asarray(A, dtype=np.float64)
    det = float(np.linalg.det(A))
    if A.shape != (3, 3) or not det > 0.0:
        raise ValueError("A must be a 3x3 matrix with positive determinant")
    cof = det * np.linalg.inv(A)             # rows: S' = S @ cof
    return BoxMesh(
        n_cells=mesh.n_cells, n_faces=mesh.n_faces, owner=mesh.owner.copy(),
        neighbour=mesh.neighbour.copy(), cell_volume=det * mesh.cell_volume,
        cell_centre=mesh.cell_centre @ A.T, face_area=mesh.face_area @ cof,
        face_centre=mesh.face_centre @ A.T, patch_names=mesh.patch_names,
        patch_start=mesh.patch_start.copy(), bface_cell=mesh.bface_cell.copy(),
        bface_area=mesh.bface_area @ cof, bface_centre=mesh.bface_centre @ A.T,
        shape=mesh.shape, ijk=mesh.ijk, nodes=None)


SKEW = ((1.0, 0.30, 0.10), (0.20, 1.0, 0.25), (-0.10, 0.15, 1.0))

# x sheared by 25 y: the x and y faces of a box make an angle of about 87.7
# degrees with the lines joining their cell centres (cosine 1/sqrt(626), below
# 1/20), the z faces stay orthogonal to them
STEEP = ((1.0, 25.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


def from_arrays(cell_centre, cell_volume, faces, patches) -> BoxMesh:
    """A mesh given face by face (small hand-made cases).

    faces: [(owner, neighbour, S_f, C_f)] in upper-triangular order;
    patches: [[(cell, S_b, C_b), ...], ...] one list of boundary faces per patch.
    """
    cc = np.asarray(cell_centre, dtype=np.float64).reshape(-1, 3)
    bf = [b for p in patches for b in p]
    starts = np.concatenate(([0], np.cumsum([len(p) for p in patches]))).astype(np.int32)
    f3 = lambda rows: np.asarray(rows, dtype=np.float64).reshape(-1, 3)
    return BoxMesh(
        n_cells=cc.shape[0], n_faces=len(faces),
        owner=np.asarray([f[0] for f in faces], dtype=np.int32),
        neighbour=np.asarray([f[1] for f in faces], dtype=np.int32),
        cell_volume=np.asarray(cell_volume, dtype=np.float64), cell_centre=cc,
        face_area=f3([f[2] for f in faces]), face_centre=f3([f[3] for f in faces]),
        patch_names=tuple(f"patch{i}" for i in range(len(patches))), patch_start=starts,
        bface_cell=np.asarray([b[0] for b in bf], dtype=np.int32),
        bface_area=f3([b[1] for b in bf]), bface_centre=f3([b[2] for b in bf]))


def box_aggregation(shape, coarsest: int = 512, min_side: int = 3):
    """Aggregation hierarchy of a box numbered c = i + nx (j + ny k): each level's
    cells grouped in 2 x 2 x 2 blocks (a direction of odd length ends with a
    block of one cell in it), coarse cells numbered the same way on the halved
    box.  Levels are added while the current one has more than `coarsest`
    cells and every side is at least `min_side` long (so that with the default
    3 every level stays a box of sides 2 or more).  Returns (level_cells,
    aggs): cells per level, and per level but the last the coarse cell of each
    of its cells."""
    nx, ny, nz = (int(v) for v in shape)
    cells = [nx * ny * nz]
    aggs = []
    while cells[-1] > coarsest and min(nx, ny, nz) >= min_side and max(nx, ny, nz) > 1:
        cx, cy, cz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
        i = np.arange(nx) // 2
        j = np.arange(ny) // 2
        k = np.arange(nz) // 2
        agg = (i[None, None, :] + cx * (j[None, :, None] + cy * k[:, None, None])).ravel()
        aggs.append(agg.astype(np.int32))
        nx, ny, nz = cx, cy, cz
        cells.append(nx * ny * nz)
    return cells, aggs


def random_permutation(n: int, seed: int) -> np.ndarray:
    """new_of_old for a seeded random relabelling: cells ranked by SplitMix64 keys."""
    keys = splitmix64(seed, n)
    order = np.argsort(keys, kind="stable")     # old labels in new order
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[order] = np.arange(n)
    return new_of_old


def red_black_numbering(mesh: BoxMesh) -> Tuple[np.ndarray, int]:
    """new_of_old putting all red cells ((i+j+k) even) first, then black.

    Both colours keep their original relative order.  Returns (new_of_old, n_red).
    On a box every internal face joins a red and a black cell, so after
    renumbering every face has a red owner and a black neighbour.
    """
    s = mesh.ijk.sum(axis=1)
    red = (s % 2) == 0
    n_red = int(red.sum())
    new_of_old = np.empty(mesh.n_cells, dtype=np.int64)
    new_of_old[np.flatnonzero(red)] = np.arange(n_red)
    new_of_old[np.flatnonzero(~red)] = n_red + np.arange(mesh.n_cells - n_red)
    return new_of_old, n_red


def initial_field(n: int, seed: int, lo: float = 273.0, hi: float = 573.0,
                  new_of_old: np.ndarray = None) -> np.ndarray:
    """T0 ~ U[lo, hi) drawn in the cell order of the unrenumbered mesh."""
    u = uniform01(seed, n)
    t = lo + (hi - lo) * u
    if new_of_old is None:
        return t
    out = np.empty_like(t)
    out[np.asarray(new_of_old)] = t
    return out


# boundary condition kinds (same integer codes as the C interface)
ZERO_GRADIENT = 0
FIXED_VALUE = 1


def fixed_x_bcs(t_lo: float = 273.0, t_hi: float = 573.0) -> List[Tuple[int, float]]:
    """fixedValue at x = 0 and x = 1, zeroGradient on the four other sides."""
    return [(FIXED_VALUE, t_lo), (FIXED_VALUE, t_hi)] + [(ZERO_GRADIENT, 0.0)] * 4


def all_zero_gradient() -> List[Tuple[int, float]]:
    return [(ZERO_GRADIENT, 0.0)] * 6
