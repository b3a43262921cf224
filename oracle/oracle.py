"""ctypes wrapper of the C oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads ``liblforacle.so`` built from ``lforacle.c`` by ``build.py``.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblforacle.so")

PC_DIAGONAL = 0
PC_DIC = 1
BC_ZERO_GRADIENT = 0
BC_FIXED_VALUE = 1


class Stats(C.Structure):
    _fields_ = [("initial_residual", C.c_double), ("final_residual", C.c_double),
                ("n_iter", C.c_int32), ("converged", C.c_int32), ("singular", C.c_int32),
                ("pad", C.c_int32), ("assemble_s", C.c_double), ("solve_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
    return _lib


def _p(a, dtype):
    assert a.dtype == dtype and a.flags.c_contiguous, (a.dtype, dtype)
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def face_geometry(mesh):
    F = mesh.n_faces
    mag = np.empty(F)
    dlt = np.empty(F)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    cc, sf = _f64(mesh.cell_centre), _f64(mesh.face_area)
    lib().lfo_face_geometry(C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                            _p(cc, np.float64), _p(sf, np.float64), _p(mag, np.float64),
                            _p(dlt, np.float64))
    return mag, dlt


def bface_geometry(mesh):
    B = mesh.n_bfaces
    mag = np.empty(B)
    dlt = np.empty(B)
    bc_ = _i32(mesh.bface_cell)
    cc, ba, bcn = _f64(mesh.cell_centre), _f64(mesh.bface_area), _f64(mesh.bface_centre)
    lib().lfo_bface_geometry(C.c_int32(B), _p(bc_, np.int32), _p(cc, np.float64),
                             _p(ba, np.float64), _p(bcn, np.float64), _p(mag, np.float64),
                             _p(dlt, np.float64))
    return mag, dlt


def _patch_arrays(mesh, bcs):
    if len(bcs) != mesh.n_patches:
        raise ValueError("one boundary condition per patch is required")
    types = np.asarray([int(t) for t, _ in bcs], dtype=np.int32)
    vals = np.asarray([float(v) for _, v in bcs], dtype=np.float64)
    return _i32(mesh.patch_start), types, vals


def assemble(mesh, bcs, DT, dt, T_old, lap_src=None):
    """Return dict with diag, upper, source, diag_b, source_b, int_coeff, bou_coeff.
    lap_src: the laplacian's explicit non-orthogonal source (None = none)."""
    N, F, B = mesh.n_cells, mesh.n_faces, mesh.n_bfaces
    mag, dlt = face_geometry(mesh)
    bmag, bdlt = bface_geometry(mesh)
    ps, pt, pv = _patch_arrays(mesh, bcs)
    out = {k: np.empty(N) for k in ("diag", "source", "diag_b", "source_b")}
    out["upper"] = np.empty(F)
    out["int_coeff"] = np.empty(B)
    out["bou_coeff"] = np.empty(B)
    own, nei, vol = _i32(mesh.owner), _i32(mesh.neighbour), _f64(mesh.cell_volume)
    bcell = _i32(mesh.bface_cell)
    T_old = _f64(T_old)
    ls = None if lap_src is None else _f64(lap_src)
    rc = lib().lfo_assemble(
        C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32), _p(vol, np.float64),
        _p(mag, np.float64), _p(dlt, np.float64), C.c_int32(mesh.n_patches), _p(ps, np.int32),
        _p(pt, np.int32), _p(pv, np.float64), _p(bcell, np.int32), _p(bmag, np.float64),
        _p(bdlt, np.float64), C.c_double(DT), C.c_double(dt), _p(T_old, np.float64),
        None if ls is None else _p(ls, np.float64), _p(out["diag"], np.float64), _p(out["upper"], np.float64), _p(out["source"], np.float64),
        _p(out["diag_b"], np.float64), _p(out["source_b"], np.float64),
        _p(out["int_coeff"], np.float64), _p(out["bou_coeff"], np.float64))
    if rc != 0:
        raise ValueError(f"oracle assemble failed: {rc}")
    return out


def amul(mesh, diag, upper, x):
    N, F = mesh.n_cells, mesh.n_faces
    y = np.empty(N)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper, x = _f64(diag), _f64(upper), _f64(x)
    lib().lfo_amul(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                   _p(diag, np.float64), _p(upper, np.float64), _p(x, np.float64),
                   _p(y, np.float64))
    return y


def sum_a(mesh, diag, upper):
    N, F = mesh.n_cells, mesh.n_faces
    y = np.empty(N)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper = _f64(diag), _f64(upper)
    lib().lfo_sum_a(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                    _p(diag, np.float64), _p(upper, np.float64), _p(y, np.float64))
    return y


def dic_rd(mesh, diag, upper):
    N, F = mesh.n_cells, mesh.n_faces
    rd = np.empty(N)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper = _f64(diag), _f64(upper)
    lib().lfo_dic_rd(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                     _p(diag, np.float64), _p(upper, np.float64), _p(rd, np.float64))
    return rd


def precondition(mesh, pc, upper, rd, r):
    N, F = mesh.n_cells, mesh.n_faces
    w = np.empty(N)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    upper, rd, r = _f64(upper), _f64(rd), _f64(r)
    lib().lfo_precondition(C.c_int(pc), C.c_int32(N), C.c_int32(F), _p(own, np.int32),
                           _p(nei, np.int32), _p(upper, np.float64), _p(rd, np.float64),
                           _p(r, np.float64), _p(w, np.float64))
    return w


def pcg(mesh, diag, upper, b, x0, pc=PC_DIAGONAL, tol=1e-9, rel_tol=0.0, max_iter=1000,
        min_iter=0):
    """Solve A x = b from x0; returns (x, stats dict)."""
    N, F = mesh.n_cells, mesh.n_faces
    x = np.array(x0, dtype=np.float64, copy=True)
    st = Stats()
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper, b = _f64(diag), _f64(upper), _f64(b)
    rc = lib().lfo_pcg(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                       _p(diag, np.float64), _p(upper, np.float64), _p(b, np.float64),
                       _p(x, np.float64), C.c_int(pc), C.c_double(tol), C.c_double(rel_tol),
                       C.c_int32(max_iter), C.c_int32(min_iter), C.byref(st))
    if rc != 0:
        raise ValueError(f"oracle pcg failed: {rc}")
    return x, st.as_dict()


def run(mesh, bcs, DT, dt, n_steps, T0, pc=PC_DIAGONAL, tol=1e-9, rel_tol=0.0, max_iter=1000,
        min_iter=0, keep_all=False):
    """Run n_steps time steps from T0.  Returns (T_final, [stats], [T per step] or None)."""
    N, F = mesh.n_cells, mesh.n_faces
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    vol, cc, sf = _f64(mesh.cell_volume), _f64(mesh.cell_centre), _f64(mesh.face_area)
    ps, pt, pv = _patch_arrays(mesh, bcs)
    bcell, ba, bcn = _i32(mesh.bface_cell), _f64(mesh.bface_area), _f64(mesh.bface_centre)
    T = np.array(T0, dtype=np.float64, copy=True)
    snaps = [] if keep_all else None
    stats_all = []
    steps_per_call = 1 if keep_all else n_steps
    done = 0
    while done < n_steps:
        k = min(steps_per_call, n_steps - done)
        st = (Stats * max(k, 1))()
        rc = lib().lfo_run(
            C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32), _p(vol, np.float64),
            _p(cc, np.float64), _p(sf, np.float64), C.c_int32(mesh.n_patches), _p(ps, np.int32),
            _p(pt, np.int32), _p(pv, np.float64), _p(bcell, np.int32), _p(ba, np.float64),
            _p(bcn, np.float64), C.c_double(DT), C.c_double(dt), C.c_int32(k), C.c_int(pc),
            C.c_double(tol), C.c_double(rel_tol), C.c_int32(max_iter), C.c_int32(min_iter),
            _p(T, np.float64), st)
        if rc != 0:
            raise ValueError(f"oracle run failed: {rc}")
        stats_all.extend(s.as_dict() for s in st[:k])
        if keep_all:
            snaps.append(T.copy())
        done += k
    return T, stats_all, snaps


def interp_weights(mesh):
    """Linear interpolation weights w_f of the internal faces (needs face centres)."""
    F = mesh.n_faces
    w = np.empty(F)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    cc, sf, fc = _f64(mesh.cell_centre), _f64(mesh.face_area), _f64(mesh.face_centre)
    lib().lfo_interp_weights(C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                             _p(cc, np.float64), _p(sf, np.float64), _p(fc, np.float64),
                             _p(w, np.float64))
    return w


def interpolate(mesh, w, v):
    """Face values s_f = w_f (v_P - v_N) + v_N."""
    F = mesh.n_faces
    s = np.empty(F)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    w, v = _f64(w), _f64(v)
    lib().lfo_interpolate(C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                          _p(w, np.float64), _p(v, np.float64), _p(s, np.float64))
    return s


def boundary_values(mesh, bcs, T):
    """(T_b, snGrad_b) on the boundary faces for the patches' conditions."""
    B = mesh.n_bfaces
    _, bdlt = bface_geometry(mesh)
    ps, pt, pv = _patch_arrays(mesh, bcs)
    Tb, snb = np.empty(B), np.empty(B)
    bcell, T = _i32(mesh.bface_cell), _f64(T)
    rc = lib().lfo_boundary_values(C.c_int32(mesh.n_patches), _p(ps, np.int32), _p(pt, np.int32),
                                   _p(pv, np.float64), _p(bcell, np.int32), _p(bdlt, np.float64),
                                   _p(T, np.float64), _p(Tb, np.float64), _p(snb, np.float64))
    if rc != 0:
        raise ValueError(f"oracle boundary_values failed: {rc}")
    return Tb, snb


def gauss_grad(mesh, T, Tb, snb, w=None):
    """Gauss gradient of the cell field T with boundary values Tb and boundary
    normal gradients snb: returns (grad [N,3], bgrad [B,3])."""
    N, F, B = mesh.n_cells, mesh.n_faces, mesh.n_bfaces
    if w is None:
        w = interp_weights(mesh)
    s = interpolate(mesh, w, T)
    grad = np.empty((N, 3))
    bgrad = np.empty((B, 3))
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    vol, sf = _f64(mesh.cell_volume), _f64(mesh.face_area)
    bcell, ba = _i32(mesh.bface_cell), _f64(mesh.bface_area)
    Tb, snb = _f64(Tb), _f64(snb)
    lib().lfo_gauss_grad(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                         _p(vol, np.float64), _p(sf, np.float64), _p(s, np.float64), C.c_int32(B),
                         _p(bcell, np.int32), _p(ba, np.float64), _p(Tb, np.float64),
                         _p(snb, np.float64), _p(grad, np.float64), _p(bgrad, np.float64))
    return grad, bgrad


def nonorth_source(mesh, DT, grad, w=None):
    """The laplacian's explicit non-orthogonal source lap_src [N] from the cell
    gradient grad [N,3] (TEqn subtracts it from its source)."""
    N, F = mesh.n_cells, mesh.n_faces
    if w is None:
        w = interp_weights(mesh)
    mag, dlt = face_geometry(mesh)
    out = np.empty(N)
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    vol, cc, sf = _f64(mesh.cell_volume), _f64(mesh.cell_centre), _f64(mesh.face_area)
    w, g = _f64(w), _f64(grad)
    rc = lib().lfo_nonorth_source(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                                  _p(vol, np.float64), _p(cc, np.float64), _p(sf, np.float64),
                                  _p(mag, np.float64), _p(dlt, np.float64), _p(w, np.float64),
                                  _p(g, np.float64), C.c_double(DT), _p(out, np.float64))
    if rc != 0:
        raise ValueError(f"oracle nonorth_source failed: {rc}")
    return out


def step_source(mesh, bcs, DT, T):
    """lap_src of a time step on a mesh with non-orthogonal faces: the
    gradient of T with its boundary values, then the correction."""
    Tb, snb = boundary_values(mesh, bcs, T)
    g, _ = gauss_grad(mesh, T, Tb, snb)
    return nonorth_source(mesh, DT, g)


def run_nonorth(mesh, bcs, DT, dt, n_steps, T0, pc=PC_DIAGONAL, tol=1e-9, rel_tol=0.0,
                max_iter=1000, min_iter=0, n_corr=0):
    """Time steps with the explicit non-orthogonal correction: per step,
    1 + n_corr passes of the corrector loop (Section 5.1), each assembling
    TEqn with its ddt source from T at the start of the step and its
    correction from the latest T, then solving from the latest T.  Returns
    (T_final, [stats per step: iterations summed over the passes, the first
    pass's initial and the last pass's final residual], [T per step])."""
    T = np.array(T0, dtype=np.float64, copy=True)
    stats, snaps = [], []
    for _ in range(n_steps):
        T_old = T.copy()
        total = None
        for _ in range(1 + n_corr):
            A = assemble(mesh, bcs, DT, dt, T_old, lap_src=step_source(mesh, bcs, DT, T))
            T, st = pcg(mesh, A["diag_b"], A["upper"], A["source_b"], T, pc=pc, tol=tol,
                        rel_tol=rel_tol, max_iter=max_iter, min_iter=min_iter)
            if total is None:
                total = dict(st)
            else:
                total.update(final_residual=st["final_residual"], converged=st["converged"],
                             singular=st["singular"], n_iter=total["n_iter"] + st["n_iter"])
        stats.append(total)
        snaps.append(T.copy())
    return T, stats, snaps


# aggregation multigrid (READING of the oracle's header): sweeps and weight
AMG_NU, AMG_NU_C, AMG_OMEGA = 2, 4, 0.8


def galerkin(n, owner, neighbour, diag, upper, agg, nc):
    """Galerkin coarse matrix P^T A P of an LDU matrix for an aggregation
    agg[n] into nc cells: (coarse owner, neighbour, diag, upper)."""
    nf = len(owner)
    own, nei = _i32(owner), _i32(neighbour)
    diag, upper, agg = _f64(diag), _f64(upper), _i32(agg)
    cap = max(nf, 1)
    co, cn = np.empty(cap, np.int32), np.empty(cap, np.int32)
    cd, cu = np.empty(nc), np.empty(cap)
    nfc = C.c_int32(0)
    rc = lib().lfo_galerkin(C.c_int32(n), C.c_int32(nf), _p(own, np.int32), _p(nei, np.int32),
                            _p(diag, np.float64), _p(upper, np.float64), _p(agg, np.int32),
                            C.c_int32(nc), C.byref(nfc), _p(co, np.int32), _p(cn, np.int32),
                            _p(cd, np.float64), _p(cu, np.float64))
    if rc != 0:
        raise ValueError(f"oracle galerkin failed: {rc}")
    k = nfc.value
    return co[:k].copy(), cn[:k].copy(), cd, cu[:k].copy()


def _levels(level_cells, aggs):
    lc = np.ascontiguousarray(level_cells, dtype=np.int32)
    ag = np.ascontiguousarray(np.concatenate(aggs) if aggs else np.zeros(1), dtype=np.int32)
    return lc, ag


def amg_apply(mesh, diag, upper, r, level_cells, aggs, nu=AMG_NU, nu_c=AMG_NU_C, omega=AMG_OMEGA):
    """One cycle of the aggregation multigrid preconditioner: w = M r."""
    N, F = mesh.n_cells, mesh.n_faces
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper, r = _f64(diag), _f64(upper), _f64(r)
    lc, ag = _levels(level_cells, aggs)
    w = np.empty(N)
    rc = lib().lfo_amg_apply(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                             _p(diag, np.float64), _p(upper, np.float64), C.c_int32(len(lc)),
                             _p(lc, np.int32), _p(ag, np.int32), C.c_int32(nu), C.c_int32(nu_c),
                             C.c_double(omega), _p(r, np.float64), _p(w, np.float64))
    if rc != 0:
        raise ValueError(f"oracle amg_apply failed: {rc}")
    return w


def pcg_amg(mesh, diag, upper, b, x0, level_cells, aggs, tol=1e-9, rel_tol=0.0, max_iter=1000,
            min_iter=0, nu=AMG_NU, nu_c=AMG_NU_C, omega=AMG_OMEGA):
    """PCG preconditioned by the aggregation multigrid cycle; returns (x, stats)."""
    N, F = mesh.n_cells, mesh.n_faces
    x = np.array(x0, dtype=np.float64, copy=True)
    st = Stats()
    own, nei = _i32(mesh.owner), _i32(mesh.neighbour)
    diag, upper, b = _f64(diag), _f64(upper), _f64(b)
    lc, ag = _levels(level_cells, aggs)
    rc = lib().lfo_pcg_amg(C.c_int32(N), C.c_int32(F), _p(own, np.int32), _p(nei, np.int32),
                           _p(diag, np.float64), _p(upper, np.float64), _p(b, np.float64),
                           _p(x, np.float64), C.c_int32(len(lc)), _p(lc, np.int32), _p(ag, np.int32),
                           C.c_int32(nu), C.c_int32(nu_c), C.c_double(omega), C.c_double(tol),
                           C.c_double(rel_tol), C.c_int32(max_iter), C.c_int32(min_iter), C.byref(st))
    if rc != 0:
        raise ValueError(f"oracle pcg_amg failed: {rc}")
    return x, st.as_dict()


def run_amg(mesh, bcs, DT, dt, n_steps, T0, level_cells, aggs, tol=1e-9, rel_tol=0.0,
            max_iter=1000, min_iter=0, keep_all=False, **kw):
    """Time steps solved by PCG with the multigrid cycle: (T_final, [stats], [T per step])."""
    T = np.array(T0, dtype=np.float64, copy=True)
    stats, snaps = [], ([] if keep_all else None)
    for _ in range(n_steps):
        A = assemble(mesh, bcs, DT, dt, T)
        T, st = pcg_amg(mesh, A["diag_b"], A["upper"], A["source_b"], T, level_cells, aggs, tol=tol,
                        rel_tol=rel_tol, max_iter=max_iter, min_iter=min_iter, **kw)
        stats.append(st)
        if keep_all:
            snaps.append(T.copy())
    return T, stats, snaps
