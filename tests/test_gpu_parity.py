"""GPU path vs the oracle, element by element, through the C ABI.

Bars: integer addressing bit-exact; assembled coefficients within 1e-14
relative; T within 1e-8 max relative error at every step; PCG iterations
within +-1; Amul bitwise when fed the same matrix (same operation order, no
FMA contraction on either side).
"""
import numpy as np
import pytest

import synth
from synth import FIXED_VALUE, ZERO_GRADIENT
from tests.gpu_common import lapfoam, run_gpu, max_rel

pytestmark = pytest.mark.gpu

COEF_TOL = 1e-14
T_TOL = 1e-8


@pytest.fixture(scope="module")
def L():
    return lapfoam()


def _meshes():
    base = synth.box_mesh(7, 5, 3, z_ratio=4.0)                 # 105 cells: ragged tail
    yield "natural_7x5x3", base
    yield "random_7x5x3", synth.renumber(base, synth.random_permutation(base.n_cells, 2))
    yield "redblack_6x6x4", synth.renumber(synth.box_mesh(6, 6, 4),
                                           synth.red_black_numbering(synth.box_mesh(6, 6, 4))[0])
    tiny = synth.box_mesh(3, 3, 2)                                # 18 cells: one partial slice
    yield "random_3x3x2", synth.renumber(tiny, synth.random_permutation(tiny.n_cells, 4))
    yield "line_9", synth.box_mesh(9, 1, 1)
    yield "one_cell", synth.box_mesh(1, 1, 1)
    g = synth.box_mesh(24, 20, 18, z_ratio=10.0)                 # several workgroups
    yield "graded_24x20x18", g
    yield "random_24x20x18", synth.renumber(g, synth.random_permutation(g.n_cells, 1))


@pytest.mark.parametrize("name,mesh", list(_meshes()), ids=[n for n, _ in _meshes()])
def test_addressing_is_exact(L, name, mesh):
    """Section 5.2 lists of lists against their definitions (bit-exact)."""
    m = L.Mesh(mesh)
    a = m.addressing()
    N = mesh.n_cells
    own, nei = mesh.owner.astype(np.int64), mesh.neighbour.astype(np.int64)
    assert np.array_equal(a["owner_start"], np.searchsorted(own, np.arange(N + 1), side="left"))
    assert np.array_equal(a["losort"], np.argsort(nei, kind="stable"))
    assert np.array_equal(a["losort_start"],
                          np.concatenate(([0], np.cumsum(np.bincount(nei, minlength=N)))))
    bc = mesh.bface_cell.astype(np.int64)
    assert np.array_equal(a["bface_list"], np.argsort(bc, kind="stable"))
    assert np.array_equal(a["bface_start"],
                          np.concatenate(([0], np.cumsum(np.bincount(bc, minlength=N)))))
    m.close()


BCS_MIXED = [(FIXED_VALUE, 273.0), (FIXED_VALUE, 573.0), (ZERO_GRADIENT, 0.0),
             (FIXED_VALUE, 400.0), (ZERO_GRADIENT, 0.0), (FIXED_VALUE, 300.0)]


def _expected_layout(mesh, layout):
    """Band layout when asked for (or AUTO) and the faces take at most 4 offsets."""
    offsets = np.unique(mesh.neighbour.astype(np.int64) - mesh.owner)
    banded = mesh.n_faces > 0 and offsets.size <= 4
    return 2 if (layout != 1 and banded) else 1


LAYOUTS = [0, 1]   # AUTO (bands where the mesh allows), ROWS


@pytest.mark.parametrize("layout", LAYOUTS, ids=["auto", "rows"])
@pytest.mark.parametrize("name,mesh", list(_meshes()), ids=[n for n, _ in _meshes()])
def test_matrix_matches_oracle(L, oracle, name, mesh, layout):
    T0 = synth.initial_field(mesh.n_cells, 5)
    DT, dt = 3e-3, 2e-3
    m = L.Mesh(mesh)
    P = L.Problem(m, BCS_MIXED, DT, dt, L.make_opts(layout=layout))
    assert P.layout() == _expected_layout(mesh, layout)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, BCS_MIXED, DT, dt, T0)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        if o[k].size == 0:
            continue
        scale = np.maximum(np.abs(o[k]), 1e-300)
        err = np.max(np.abs(g[k] - o[k]) / scale)
        assert err <= COEF_TOL, (k, err)
    P.close()
    m.close()


@pytest.mark.parametrize("layout", LAYOUTS, ids=["auto", "rows"])
def test_matrix_is_bitwise_equal_to_oracle(L, oracle, layout):
    """Same operation order and no contraction: the coefficients agree bit for bit."""
    mesh = synth.box_mesh(24, 20, 18, z_ratio=10.0)
    T0 = synth.initial_field(mesh.n_cells, 6)
    m = L.Mesh(mesh)
    P = L.Problem(m, BCS_MIXED, 1e-3, 1e-3, L.make_opts(layout=layout))
    assert P.layout() == _expected_layout(mesh, layout)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    o = oracle.assemble(mesh, BCS_MIXED, 1e-3, 1e-3, T0)
    for k in ("diag", "upper", "source", "diag_b", "source_b", "int_coeff", "bou_coeff"):
        assert np.array_equal(g[k], o[k]), k
    P.close()
    m.close()


@pytest.mark.parametrize("layout", LAYOUTS, ids=["auto", "rows"])
@pytest.mark.parametrize("name,mesh", list(_meshes()), ids=[n for n, _ in _meshes()])
def test_amul_bitwise(L, oracle, name, mesh, layout):
    import torch
    T0 = synth.initial_field(mesh.n_cells, 7)
    m = L.Mesh(mesh)
    P = L.Problem(m, BCS_MIXED, 1e-3, 1e-3, L.make_opts(layout=layout))
    assert P.layout() == _expected_layout(mesh, layout)
    P.set_T(T0)
    P.assemble()
    g = P.matrix()
    x = np.random.default_rng(3).uniform(-1.0, 1.0, mesh.n_cells)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    P.amul(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    y_ref = oracle.amul(mesh, g["diag_b"], g["upper"], x)
    assert np.array_equal(y, y_ref)
    P.close()
    m.close()


WALK_MESHES = [
    # band-1 offset d1 = nx; runs of 8 d1 rows, the last one ragged
    ("13x7x5", lambda: synth.box_mesh(13, 7, 5, z_ratio=3.0)),
    ("5x40x9", lambda: synth.box_mesh(5, 40, 9, z_ratio=2.0)),
    ("two_bands_6x5x1", lambda: synth.box_mesh(6, 5, 1)),
    ("one_plane_row_3x1x7", lambda: synth.box_mesh(3, 1, 7)),
    # block walk (nx even): tiles of 2 lines x 2 planes, nx / 2 threads each
    ("block_130x9x4", lambda: synth.box_mesh(130, 9, 4)),          # tiles cross waves, odd line count
    ("block_2x7x5", lambda: synth.box_mesh(2, 7, 5, z_ratio=2.0)),  # one thread per tile, odd lines and planes
    ("block_128x6x3", lambda: synth.box_mesh(128, 6, 3)),           # one wave per tile line, odd planes
    ("block_256x3x2", lambda: synth.box_mesh(256, 3, 2, z_ratio=4.0)),  # two waves per line
    ("block_66x5x7", lambda: synth.box_mesh(66, 5, 7, z_ratio=3.0)),
]


def _block_form(name):
    """The meshes above on which LF_WALK_ON takes the block walk."""
    return name.startswith("block_")


@pytest.mark.parametrize("name,mk", WALK_MESHES, ids=[n for n, _ in WALK_MESHES])
def test_amul_walk_bitwise(L, oracle, name, mk):
    """The row-walk product equals the one-row-per-thread product and the
    oracle's LDU product bitwise (same terms in the same order)."""
    import torch
    mesh = mk()
    T0 = synth.initial_field(mesh.n_cells, 8)
    x = np.random.default_rng(4).uniform(-1.0, 1.0, mesh.n_cells)
    m = L.Mesh(mesh)
    assert m.n_bands >= 2
    ys = []
    for walk in (L.LF_WALK_ON, L.LF_WALK_OFF):
        P = L.Problem(m, BCS_MIXED, 2e-3, 1e-3, L.make_opts(amul_walk=walk))
        assert P.layout() == L.LF_LAYOUT_BANDS
        assert P.amul_walk() == (walk == L.LF_WALK_ON)
        if walk == L.LF_WALK_ON:
            assert P.amul_form() == (2 if _block_form(name) else 1), P.amul_form()
        P.set_T(T0)
        P.assemble()
        g = P.matrix()
        xd = torch.from_numpy(x).cuda()
        yd = torch.empty_like(xd)
        P.amul(xd, yd)
        torch.cuda.synchronize()
        ys.append(yd.cpu().numpy())
        P.close()
    assert np.array_equal(ys[0], ys[1])
    assert np.array_equal(ys[0], oracle.amul(mesh, g["diag_b"], g["upper"], x))
    m.close()


def _morton(C):
    """Z-order keys of points, 21 bits per axis over their bounding box."""
    lo, hi = C.min(axis=0), C.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.floor(np.clip((C - lo) / span, 0.0, 1.0) * 2097151.0).astype(np.uint64)
    key = np.zeros(len(C), dtype=np.uint64)
    for bit in range(21):
        for k in range(3):
            key |= ((q[:, k] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + k)
    return key


def test_cell_order():
    """Meshes without band form and without two colours are kept in Morton
    order of their cell centres (a permutation, keys nondecreasing, ties by
    index); structured and red-black numberings keep their own order."""
    L = lapfoam()
    base = synth.box_mesh(9, 7, 5, z_ratio=3.0)
    rnd = synth.renumber(base, synth.random_permutation(base.n_cells, 8))
    m = L.Mesh(rnd)
    reordered, order = m.cell_order()
    assert reordered
    assert np.array_equal(np.sort(order), np.arange(rnd.n_cells))
    key = _morton(rnd.cell_centre.reshape(-1, 3))[order]
    assert np.all((key[1:] > key[:-1]) | ((key[1:] == key[:-1]) & (order[1:] > order[:-1])))
    m.close()
    for mesh in (base, synth.renumber(synth.box_mesh(6, 6, 4),
                                      synth.red_black_numbering(synth.box_mesh(6, 6, 4))[0])):
        m = L.Mesh(mesh)
        reordered, order = m.cell_order()
        assert not reordered and np.array_equal(order, np.arange(mesh.n_cells))
        m.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_step_begin_poll_equals_step(L, precision):
    """lf_step_begin / lf_step_poll: bitwise the snapshots and stats of stepping
    one step at a time, snapshots in the mesh's cell order (also on a mesh the
    solver keeps in Morton order); the problem refuses other calls while the
    run is in flight."""
    import torch
    base = synth.box_mesh(12, 10, 9, z_ratio=3.0)
    meshes = [base, synth.renumber(base, synth.random_permutation(base.n_cells, 3))]
    steps = 4
    for mesh in meshes:
        N = mesh.n_cells
        T0 = synth.initial_field(N, 31)
        m = L.Mesh(mesh)
        opts = L.make_opts(precision=precision)
        A = L.Problem(m, BCS_MIXED, 5e-3, 2e-3, opts)
        A.set_T(T0)
        ref, sref = [], []
        for _ in range(steps):
            st, _ = A.step(1)
            sref += st
            ref.append(A.get_T())
        B = L.Problem(m, BCS_MIXED, 5e-3, 2e-3, opts)
        B.set_T(T0)
        with pytest.raises(L.LapfoamError):
            B.step_poll()                                # nothing started
        snap = torch.empty(steps * N, dtype=torch.float64, device="cuda")
        B.step_begin(steps, snap)
        with pytest.raises(L.LapfoamError):
            B.step(1)                                    # a run is in flight
        with pytest.raises(L.LapfoamError):
            B.get_T()
        while True:
            done, finished, stats, status = B.step_poll()
            if finished:
                break
        assert status == L.LF_OK and done == steps
        got = snap.view(steps, N).cpu().numpy()
        for s in range(steps):
            assert np.array_equal(got[s], ref[s]), s
            assert stats[s]["n_iter"] == sref[s]["n_iter"]
            assert stats[s]["final_residual"] == sref[s]["final_residual"]
        assert np.array_equal(B.get_T(), ref[-1])
        A.close()
        B.close()
        m.close()


def test_amul_walk_option_checked(L):
    m = L.Mesh(synth.box_mesh(4, 4, 4))
    with pytest.raises(L.LapfoamError):
        L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(amul_walk=7))
    # rows layout and one-band meshes keep the one-row-per-thread product
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(layout=1, amul_walk=L.LF_WALK_ON))
    assert not P.amul_walk()
    P.close()
    m.close()
    m = L.Mesh(synth.box_mesh(9, 1, 1))
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(amul_walk=L.LF_WALK_ON))
    assert not P.amul_walk()
    P.close()
    m.close()


CASES = [
    # name, config, n override, steps, precond
    ("plain_32", "plain_32", None, 20, 0),
    ("graded_24", "graded_256", 24, 6, 0),
    ("permuted_20", "permuted_192", 20, 6, 0),
    ("dic_redblack_16", "graded_256_dic", 16, 6, 1),
    ("dic_redblack_odd_9", "graded_256_dic", 9, 4, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_steps_match_oracle(L, oracle, case):
    name, cfg, n, steps, pc = case
    p = synth.build_config(cfg, n=n, steps=steps)
    Tg, sg = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, steps, precond=pc)
    To, so, snaps = oracle.run(p.mesh, p.bcs, p.DT, p.dt, steps, p.T0, pc=pc, keep_all=True)
    for s in range(steps):
        assert max_rel(Tg[s], snaps[s]) <= T_TOL, (s, max_rel(Tg[s], snaps[s]))
        assert abs(sg[s]["n_iter"] - so[s]["n_iter"]) <= 1, (s, sg[s], so[s])
        assert sg[s]["converged"] == 1 and so[s]["converged"] == 1
        assert abs(sg[s]["initial_residual"] - so[s]["initial_residual"]) <= \
            1e-10 * so[s]["initial_residual"]
        assert sg[s]["final_residual"] < 1e-9
        assert sg[s]["singular"] == 0 and sg[s]["nonfinite"] == 0


EDGE = [
    ("one_cell", lambda: synth.box_mesh(1, 1, 1, lengths=(0.5, 0.25, 2.0)), synth.fixed_x_bcs(), 0.7, 0.3, {}),
    ("two_cells", lambda: synth.box_mesh(2, 1, 1), synth.fixed_x_bcs(), 0.2, 0.1, {}),
    ("line_33", lambda: synth.box_mesh(33, 1, 1), synth.fixed_x_bcs(), 0.05, 0.01, {}),
    ("all_zero_gradient", lambda: synth.box_mesh(9, 7, 5, z_ratio=3.0), synth.all_zero_gradient(), 1e-2, 1e-2, {}),
    ("zero_DT", lambda: synth.box_mesh(8, 8, 8), synth.fixed_x_bcs(), 0.0, 1e-3, {}),
    ("max_iter_1", lambda: synth.box_mesh(10, 10, 10), synth.fixed_x_bcs(), 1e-2, 1e-2, dict(max_iter=1)),
    ("min_iter_7", lambda: synth.box_mesh(10, 10, 10), synth.fixed_x_bcs(), 1e-3, 1e-3, dict(min_iter=7)),
    ("rel_tol", lambda: synth.box_mesh(10, 10, 10), synth.fixed_x_bcs(), 1e-2, 1e-2, dict(rel_tol=1e-3)),
    ("rows_layout", lambda: synth.box_mesh(13, 11, 9, z_ratio=2.0), synth.fixed_x_bcs(), 1e-2, 1e-2,
     dict(layout=1)),
    ("bands_layout", lambda: synth.box_mesh(13, 11, 9, z_ratio=2.0), synth.fixed_x_bcs(), 1e-2, 1e-2,
     dict(layout=2)),
    ("walk_13x11x9", lambda: synth.box_mesh(13, 11, 9, z_ratio=2.0), synth.fixed_x_bcs(), 1e-2, 1e-2,
     dict(amul_walk=1)),
    ("walk_130x9x4", lambda: synth.box_mesh(130, 9, 4), synth.fixed_x_bcs(), 1e-2, 1e-2, dict(amul_walk=1)),
    ("block_walk_66x5x7", lambda: synth.box_mesh(66, 5, 7, z_ratio=3.0), synth.fixed_x_bcs(), 1e-2, 1e-2,
     dict(amul_walk=1)),
    ("block_walk_2x7x5", lambda: synth.box_mesh(2, 7, 5), synth.fixed_x_bcs(), 1e-2, 1e-2, dict(amul_walk=1)),
    ("walk_min_iter_5", lambda: synth.box_mesh(13, 11, 9), synth.fixed_x_bcs(), 1e-3, 1e-3,
     dict(amul_walk=1, min_iter=5)),
    ("no_graph", lambda: synth.box_mesh(13, 11, 9), synth.fixed_x_bcs(), 1e-2, 1e-2, dict(use_graph=0)),
    ("check_every_iter", lambda: synth.box_mesh(13, 11, 9), synth.fixed_x_bcs(), 1e-2, 1e-2,
     dict(iters_per_check=1)),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
def test_edge_cases_match_oracle(L, oracle, case):
    name, mk, bcs, DT, dt, opts = case
    mesh = mk()
    T0 = synth.initial_field(mesh.n_cells, 13)
    steps = 3
    oo = {k: v for k, v in opts.items() if k in ("max_iter", "min_iter", "rel_tol")}
    Tg, sg = run_gpu(L, mesh, bcs, DT, dt, T0, steps, **opts)
    To, so, snaps = oracle.run(mesh, bcs, DT, dt, steps, T0, keep_all=True, **oo)
    for s in range(steps):
        assert max_rel(Tg[s], snaps[s]) <= T_TOL, (name, s)
        assert abs(sg[s]["n_iter"] - so[s]["n_iter"]) <= 1, (name, s, sg[s], so[s])
        assert sg[s]["converged"] == so[s]["converged"], (name, s, sg[s], so[s])
    if name == "zero_DT":
        assert all(s["n_iter"] == 0 for s in sg)
    if name == "max_iter_1":
        assert all(s["n_iter"] == 1 and s["converged"] == 0 for s in sg)
    if name == "min_iter_7":
        assert all(s["n_iter"] >= 7 for s in sg)


@pytest.mark.parametrize("n", [6, 72], ids=["folded_reductions_6", "finalize_kernels_72"])
def test_singular_break_matches_oracle(L, oracle, n):
    """T0 = 0 with all walls zeroGradient gives r0 = 0 exactly; minIter = 1 forces
    one iteration, whose direction is 0: p.Ap = 0 breaks the loop as singular,
    no iteration counted, T unchanged.  6^3 takes the iteration's decisions
    inside the update and direction kernels, 72^3 in the one-workgroup
    finalize kernels."""
    mesh = synth.box_mesh(n, n, n)
    T0 = np.zeros(mesh.n_cells)
    Tg, sg = run_gpu(L, mesh, synth.all_zero_gradient(), 1e-3, 1e-3, T0, 2, min_iter=1)
    _, so, _ = oracle.run(mesh, synth.all_zero_gradient(), 1e-3, 1e-3, 2, T0, keep_all=True, min_iter=1)
    for s in range(2):
        assert so[s]["singular"] == 1 and so[s]["n_iter"] == 0
        assert sg[s]["singular"] == 1 and sg[s]["n_iter"] == 0, sg[s]
        assert sg[s]["nonfinite"] == 0
        assert np.array_equal(Tg[s], T0)


def test_determinism_and_graph_equivalence(L):
    """No atomics in floating point: two runs, with or without graphs, are bitwise equal."""
    p = synth.build_config("permuted_192", n=22, steps=4)
    a, sa = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 4)
    b, sb = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 4)
    c, sc = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 4, use_graph=0, iters_per_check=3)
    for s in range(4):
        assert np.array_equal(a[s], b[s]) and np.array_equal(a[s], c[s])
        for k in ("n_iter", "initial_residual", "final_residual"):
            assert sa[s][k] == sb[s][k] == sc[s][k]


def test_multi_step_call_equals_single_steps(L):
    p = synth.build_config("graded_256", n=16, steps=5)
    a, _ = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 5)
    b, _ = run_gpu(L, p.mesh, p.bcs, p.DT, p.dt, p.T0, 5, keep_all=False)
    assert np.array_equal(a[-1], b[-1])


def test_set_T_rejects_nonfinite(L):
    import torch
    mesh = synth.box_mesh(4, 4, 4)
    m = L.Mesh(mesh)
    P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3)
    bad = np.full(mesh.n_cells, 300.0)
    bad[5] = np.nan
    with pytest.raises(L.LapfoamError):
        P.set_T(bad)
    bad_d = torch.from_numpy(bad).cuda()
    with pytest.raises(L.LapfoamError):
        P.set_T(bad_d)
    P.set_T(torch.full((mesh.n_cells,), 300.0, dtype=torch.float64, device="cuda"))
    assert np.all(P.get_T() == 300.0)
    P.close()
    m.close()


def test_dic_refused_without_two_colours(L):
    mesh = synth.box_mesh(4, 4, 4)
    m = L.Mesh(mesh)
    with pytest.raises(L.LapfoamError) as e:
        L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(precond=L.LF_PC_DIC))
    assert e.value.status == L.LF_EINVAL
    m.close()


def test_problem_reset_equals_fresh_problem(L, oracle):
    """lf_problem_reset re-targets a problem (BCs, DT, dt): its steps are bitwise
    those of a problem created with the new values, in both precision forms."""
    mesh = synth.box_mesh(12, 10, 9, z_ratio=3.0)
    m = L.Mesh(mesh)
    T0 = synth.initial_field(mesh.n_cells, 21)
    bcs2 = [(FIXED_VALUE, 300.0), (ZERO_GRADIENT, 0.0), (FIXED_VALUE, 450.0), (ZERO_GRADIENT, 0.0),
            (ZERO_GRADIENT, 0.0), (FIXED_VALUE, 350.0)]
    for precision in (L.LF_PREC_FP64, L.LF_PREC_MIXED):
        P = L.Problem(m, synth.fixed_x_bcs(), 1e-3, 1e-3, L.make_opts(precision=precision))
        P.set_T(T0)
        P.step(2)
        P.reset(bcs2, 5e-3, 2e-3)
        P.set_T(T0)
        s1 = []
        for _ in range(3):
            # each step against the oracle's step from the same T (the per-step bar)
            T_prev = P.get_T()
            st, _ = P.step(1)
            s1 += st
            ref, _, _ = oracle.run(mesh, bcs2, 5e-3, 2e-3, 1, T_prev)
            assert max_rel(P.get_T(), ref) <= T_TOL, (precision, max_rel(P.get_T(), ref))
        Q = L.Problem(m, bcs2, 5e-3, 2e-3, L.make_opts(precision=precision))
        Q.set_T(T0)
        s2, _ = Q.step(3)
        assert np.array_equal(P.get_T(), Q.get_T()), precision
        assert [s["n_iter"] for s in s1] == [s["n_iter"] for s in s2]
        with pytest.raises(L.LapfoamError):
            P.reset(bcs2, -1.0, 2e-3)
        P.close()
        Q.close()
    m.close()


def test_boundary_face_values(L):
    """Boundary-face field: the patch value on fixedValue patches, the cell's T on
    zeroGradient patches (boundary-face order), before and after a step."""
    mesh = synth.box_mesh(7, 5, 4, z_ratio=2.0)
    m = L.Mesh(mesh)
    P = L.Problem(m, BCS_MIXED, 1e-3, 1e-3)
    T0 = synth.initial_field(mesh.n_cells, 9)
    P.set_T(T0)
    patch_of = np.repeat(np.arange(mesh.n_patches), np.diff(mesh.patch_start))
    for T in (T0, None):
        if T is None:
            P.step(1)
            T = P.get_T()
        want = np.array([BCS_MIXED[p][1] if BCS_MIXED[p][0] == FIXED_VALUE else T[c]
                         for p, c in zip(patch_of, mesh.bface_cell)])
        assert np.array_equal(P.boundary_T(), want)
    P.close()
    m.close()


def test_step_many_equals_single_steps(L):
    """lf_step_many interleaves the solves of several problems (own streams,
    different meshes, layouts and precision forms): each result is bitwise the
    one lf_step gives for that problem alone."""
    import torch
    cases = [
        (synth.box_mesh(20, 17, 13, z_ratio=4.0), dict()),
        (synth.renumber(synth.box_mesh(11, 9, 8), synth.random_permutation(792, 3)), dict()),
        (synth.box_mesh(24, 24, 24), dict(precision=L.LF_PREC_MIXED)),
        (synth.box_mesh(16, 12, 10), dict(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_ROWS)),
    ]
    steps = 3

    def make():
        out = []
        for i, (mesh, o) in enumerate(cases):
            m = L.Mesh(mesh)
            P = L.Problem(m, BCS_MIXED, 2e-3, 1e-3, L.make_opts(**o), stream=torch.cuda.Stream())
            P.set_T(synth.initial_field(mesh.n_cells, 40 + i))
            out.append((m, P))
        return out

    alone = make()
    ref = []
    for m, P in alone:
        st, _ = P.step(steps)
        ref.append((P.get_T(), [s["n_iter"] for s in st]))
    together = make()
    stats, status = L.step_many([P for _, P in together], steps)
    assert status == L.LF_OK
    for (m, P), (T_ref, it_ref), st in zip(together, ref, stats):
        assert np.array_equal(P.get_T(), T_ref)
        assert [s["n_iter"] for s in st] == it_ref
    with pytest.raises(L.LapfoamError):
        L.step_many([together[0][1], together[0][1]], 1)        # the same problem twice
    for m, P in alone + together:
        P.close()
        m.close()


def test_calls_refused_while_in_flight_and_duplicate_batch_tasks(L):
    """While an lf_step_begin run is in flight the problem is neither assembled
    nor read through the test hooks or the boundary values, and no batch
    launch takes it (LF_ESTATE); a batch launch listing one problem twice is
    refused (LF_EINVAL).  Everything works again once the run has finished."""
    import time
    import torch
    mesh = synth.box_mesh(10, 9, 8)
    m = L.Mesh(mesh)
    P = L.Problem(m, BCS_MIXED, 5e-3, 2e-3, L.make_opts(precision=L.LF_PREC_MIXED,
                                                        layout=L.LF_LAYOUT_ROWS))
    Q = L.Problem(m, BCS_MIXED, 5e-3, 2e-3, L.make_opts(precision=L.LF_PREC_MIXED,
                                                        layout=L.LF_LAYOUT_ROWS))
    T0 = synth.initial_field(mesh.n_cells, 41)
    P.set_T(T0)
    Q.set_T(T0)
    P.assemble()
    x = torch.ones(mesh.n_cells, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    B = L.Batch(4, 2)
    with pytest.raises(L.LapfoamError, match="LF_EINVAL"):
        B.launch([Q, Q], 1)
    P.step_begin(3)
    refused = []
    for name, call in (("assemble", P.assemble), ("matrix", P.matrix),
                       ("amul", lambda: P.amul(x, y)), ("boundary_T", P.boundary_T),
                       ("batch", lambda: B.launch([Q, P], 1))):
        try:
            call()
        except L.LapfoamError as e:
            refused.append((name, "LF_ESTATE" in str(e)))
        else:
            refused.append((name, False))
    t0 = time.time()
    finished = False
    while not finished and time.time() - t0 < 60:
        _, finished, _, _ = P.step_poll()
    assert finished
    # the run advances only through step_poll, so it was in flight at each call
    assert all(ok for _, ok in refused), refused
    P.assemble()
    P.matrix()
    P.boundary_T()
    B.launch([Q, P], 1)
    B.wait()
    B.close()
    P.close()
    Q.close()
    m.close()
