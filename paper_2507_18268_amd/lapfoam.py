"""Python binding of liblapfoam.so (the C interface declared in include/lapfoam.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (the caller-owned workspaces) and the
stream.  If the library is missing the import fails: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblapfoam.so")

LF_OK = 0
LF_EINVAL = -1
LF_EMESH = -2
LF_ENOMEM = -3
LF_EBUDGET = -4
LF_EDEVICE = -5
LF_ESTATE = -6
LF_ENONFINITE = -7

LF_BC_ZERO_GRADIENT = 0
LF_BC_FIXED_VALUE = 1
LF_PC_DIAGONAL = 0
LF_PC_DIC = 1
LF_PC_AMG = 2
LF_PREC_FP64 = 0
LF_PREC_MIXED = 1
LF_LAYOUT_AUTO = 0
LF_LAYOUT_ROWS = 1
LF_LAYOUT_BANDS = 2
LF_WALK_AUTO = 0
LF_WALK_ON = 1
LF_WALK_OFF = 2
LF_MESH_NON_ORTHOGONAL = 1

_STATUS = {0: "LF_OK", -1: "LF_EINVAL", -2: "LF_EMESH", -3: "LF_ENOMEM", -4: "LF_EBUDGET",
           -5: "LF_EDEVICE", -6: "LF_ESTATE", -7: "LF_ENONFINITE"}


class LapfoamError(RuntimeError):
    def __init__(self, status, func, msg):
        self.status = status
        super().__init__(f"{func}: {_STATUS.get(status, status)}: {msg}")


class lf_mesh_desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_faces", C.c_int32), ("n_patches", C.c_int32),
                ("flags", C.c_int32), ("owner", C.c_void_p), ("neighbour", C.c_void_p),
                ("cell_volume", C.c_void_p), ("cell_centre", C.c_void_p),
                ("face_area", C.c_void_p), ("face_centre", C.c_void_p),
                ("patch_start", C.c_void_p), ("bface_cell", C.c_void_p),
                ("bface_area", C.c_void_p), ("bface_centre", C.c_void_p)]


class lf_patch_bc(C.Structure):
    _fields_ = [("type", C.c_int32), ("reserved", C.c_int32), ("value", C.c_double)]


class lf_solver_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("rel_tol", C.c_double), ("max_iter", C.c_int32),
                ("min_iter", C.c_int32), ("precond", C.c_int32), ("precision", C.c_int32),
                ("iters_per_check", C.c_int32), ("use_graph", C.c_int32),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("layout", C.c_int32),
                ("amul_walk", C.c_int32), ("inner_restart", C.c_int32),
                ("n_nonorth_corr", C.c_int32)]


class lf_solve_stats(C.Structure):
    _fields_ = [("initial_residual", C.c_double), ("final_residual", C.c_double),
                ("n_iter", C.c_int32), ("converged", C.c_int32), ("singular", C.c_int32),
                ("nonfinite", C.c_int32), ("n_outer", C.c_int32), ("reserved", C.c_int32),
                ("assemble_ms", C.c_double), ("solve_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None

_SIGS = {
    "lf_last_error": (C.c_char_p, []),
    "lf_default_opts": (C.c_int32, [C.POINTER(lf_solver_opts)]),
    "lf_mesh_workspace_bytes": (C.c_size_t, [C.POINTER(lf_mesh_desc)]),
    "lf_mesh_create": (C.c_int32, [C.POINTER(lf_mesh_desc), C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "lf_mesh_destroy": (C.c_int32, [C.c_void_p]),
    "lf_mesh_bands": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "lf_mesh_get_addressing": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 5),
    "lf_problem_workspace_bytes": (C.c_size_t, [C.c_void_p, C.POINTER(lf_solver_opts)]),
    "lf_problem_create": (C.c_int32, [C.c_void_p, C.POINTER(lf_patch_bc), C.c_double, C.c_double,
                                      C.POINTER(lf_solver_opts), C.c_void_p, C.c_size_t,
                                      C.c_void_p, C.POINTER(C.c_void_p)]),
    "lf_problem_destroy": (C.c_int32, [C.c_void_p]),
    "lf_problem_layout": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "lf_problem_amul_walk": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "lf_mesh_cell_order": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "lf_step_begin": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lf_step_poll": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p]),
    "lf_problem_reset": (C.c_int32, [C.c_void_p, C.POINTER(lf_patch_bc), C.c_double, C.c_double]),
    "lf_set_T": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "lf_get_T": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "lf_get_boundary_T": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "lf_step": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lf_step_many": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "lf_assemble": (C.c_int32, [C.c_void_p]),
    "lf_get_matrix": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 7),
    "lf_amul": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_grad": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 5),
    "lf_grad_noalloc": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 5),
    "lf_amul_inner": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_problem_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_group_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "lf_group_create": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "lf_group_destroy": (C.c_int32, [C.c_void_p]),
    "lf_group_add": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_group_poll": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]),
    "lf_batch_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "lf_batch_create": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "lf_batch_destroy": (C.c_int32, [C.c_void_p]),
    "lf_batch_launch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_int32, C.c_int32]),
    "lf_batch_poll": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "lf_batch_wait": (C.c_int32, [C.c_void_p]),
    "lf_batch_stats": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "lf_precondition": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_profile_enable": (C.c_int32, [C.c_void_p, C.c_int32]),
    "lf_profile_read": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
}

KERNEL_CLASSES = ["assemble", "sum_x", "commit", "direction", "amul_dot", "update", "dic_rd",
                  "dic_forward", "dic_backward", "mixed_residual", "mixed_correct",
                  "inner_direction", "inner_amul_dot", "inner_update", "mixed_prep", "finalize",
                  "amg_smooth", "amg_restrict", "amg_prolong", "amg_galerkin", "grad", "nonorth",
                  "scale"]


def lib():
    """Load liblapfoam.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, func):
    if status != LF_OK:
        raise LapfoamError(status, func, lib().lf_last_error().decode())


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# same-name thin wrappers
# --------------------------------------------------------------------------
def lf_last_error():
    return lib().lf_last_error().decode()


def lf_default_opts():
    o = lf_solver_opts()
    _check(lib().lf_default_opts(C.byref(o)), "lf_default_opts")
    return o


def lf_mesh_workspace_bytes(desc):
    return int(lib().lf_mesh_workspace_bytes(C.byref(desc)))


def lf_mesh_create(desc, ws_ptr, ws_bytes, stream):
    h = C.c_void_p()
    _check(lib().lf_mesh_create(C.byref(desc), C.c_void_p(ws_ptr), C.c_size_t(ws_bytes),
                                C.c_void_p(stream), C.byref(h)), "lf_mesh_create")
    return h


def lf_mesh_destroy(h):
    _check(lib().lf_mesh_destroy(h), "lf_mesh_destroy")


def lf_mesh_bands(h):
    """(n_bands, offsets[4]) of a device mesh."""
    n = C.c_int32(0)
    offs = (C.c_int32 * 4)()
    _check(lib().lf_mesh_bands(h, C.byref(n), offs), "lf_mesh_bands")
    return n.value, list(offs)


def lf_mesh_get_addressing(h, owner_start=None, losort=None, losort_start=None,
                           bface_start=None, bface_list=None):
    _check(lib().lf_mesh_get_addressing(h, _ptr(owner_start), _ptr(losort), _ptr(losort_start),
                                        _ptr(bface_start), _ptr(bface_list)),
           "lf_mesh_get_addressing")


def lf_problem_workspace_bytes(mesh_h, opts):
    return int(lib().lf_problem_workspace_bytes(mesh_h, C.byref(opts)))


def lf_problem_create(mesh_h, bcs, DT, dt, opts, ws_ptr, ws_bytes, stream):
    h = C.c_void_p()
    _check(lib().lf_problem_create(mesh_h, bcs, C.c_double(DT), C.c_double(dt), C.byref(opts),
                                   C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream),
                                   C.byref(h)), "lf_problem_create")
    return h


def lf_problem_destroy(h):
    _check(lib().lf_problem_destroy(h), "lf_problem_destroy")


def lf_problem_reset(h, bcs_array, DT, dt):
    _check(lib().lf_problem_reset(h, bcs_array, C.c_double(DT), C.c_double(dt)), "lf_problem_reset")


def lf_problem_layout(h):
    v = C.c_int32(0)
    _check(lib().lf_problem_layout(h, C.byref(v)), "lf_problem_layout")
    return v.value


def lf_mesh_cell_order(h, n_cells):
    """(reordered, order) of a device mesh: order[r] = mesh cell of solver row r."""
    v = C.c_int32(0)
    order = np.empty(n_cells, dtype=np.int32)
    _check(lib().lf_mesh_cell_order(h, C.byref(v), order.ctypes.data), "lf_mesh_cell_order")
    return bool(v.value), order


def lf_step_begin(h, n_steps, snapshots_ptr=None):
    _check(lib().lf_step_begin(h, int(n_steps), snapshots_ptr), "lf_step_begin")


def lf_step_poll(h, n_steps):
    """(steps_done, finished, stats of the finished steps, status); status is
    LF_OK or LF_ENONFINITE (other errors raise)."""
    done, fin = C.c_int32(0), C.c_int32(0)
    st = (lf_solve_stats * max(int(n_steps), 1))()
    status = lib().lf_step_poll(h, C.byref(done), C.byref(fin), st)
    if status not in (LF_OK, LF_ENONFINITE):
        _check(status, "lf_step_poll")
    return done.value, bool(fin.value), [st[i].as_dict() for i in range(done.value)], status


def lf_problem_amul_walk(h):
    v = C.c_int32(0)
    _check(lib().lf_problem_amul_walk(h, C.byref(v)), "lf_problem_amul_walk")
    return v.value


def lf_set_T(h, ptr, on_device):
    _check(lib().lf_set_T(h, C.c_void_p(ptr), C.c_int32(on_device)), "lf_set_T")


def lf_get_T(h, ptr, on_device):
    _check(lib().lf_get_T(h, C.c_void_p(ptr), C.c_int32(on_device)), "lf_get_T")


def lf_step_many(handles, n_steps, stats_array=None):
    arr = (C.c_void_p * len(handles))(*handles)
    return lib().lf_step_many(arr, C.c_int32(len(handles)), C.c_int32(n_steps), stats_array)


def step_many(problems, n_steps=1, check=True):
    """Advance several problems together (lf_step_many); returns (per-problem
    lists of per-step stats, status)."""
    k = len(problems)
    stats = (lf_solve_stats * max(k * n_steps, 1))()
    status = lf_step_many([P.h for P in problems], n_steps, stats)
    if check:
        _check(status, "lf_step_many")
    return [[stats[i * n_steps + s].as_dict() for s in range(n_steps)] for i in range(k)], status


def lf_get_boundary_T(h, ptr, on_device):
    _check(lib().lf_get_boundary_T(h, C.c_void_p(ptr), C.c_int32(on_device)), "lf_get_boundary_T")


def lf_step(h, n_steps, stats_array=None):
    st = stats_array if stats_array is not None else None
    status = lib().lf_step(h, C.c_int32(n_steps), st)
    return status


def lf_assemble(h):
    _check(lib().lf_assemble(h), "lf_assemble")


def lf_get_matrix(h, diag=None, upper=None, source=None, diag_b=None, source_b=None,
                  int_coeff=None, bou_coeff=None):
    _check(lib().lf_get_matrix(h, _ptr(diag), _ptr(upper), _ptr(source), _ptr(diag_b),
                               _ptr(source_b), _ptr(int_coeff), _ptr(bou_coeff)),
           "lf_get_matrix")


def lf_grad(h, T_ptr, Tb_ptr, snb_ptr, grad_ptr, bgrad_ptr):
    _check(lib().lf_grad(h, C.c_void_p(T_ptr), C.c_void_p(Tb_ptr), C.c_void_p(snb_ptr),
                         C.c_void_p(grad_ptr), C.c_void_p(bgrad_ptr)), "lf_grad")


def lf_grad_noalloc(h, T_ptr, Tb_ptr, snb_ptr, grad_ptr, bgrad_ptr):
    _check(lib().lf_grad_noalloc(h, C.c_void_p(T_ptr), C.c_void_p(Tb_ptr), C.c_void_p(snb_ptr),
                                 C.c_void_p(grad_ptr), C.c_void_p(bgrad_ptr)), "lf_grad_noalloc")


def lf_problem_grad(h, grad_ptr, bgrad_ptr):
    _check(lib().lf_problem_grad(h, C.c_void_p(grad_ptr), C.c_void_p(bgrad_ptr)), "lf_problem_grad")


def lf_amul(h, x_ptr, y_ptr):
    _check(lib().lf_amul(h, C.c_void_p(x_ptr), C.c_void_p(y_ptr)), "lf_amul")


def lf_amul_inner(h, x_ptr, y_ptr):
    _check(lib().lf_amul_inner(h, C.c_void_p(x_ptr), C.c_void_p(y_ptr)), "lf_amul_inner")


def lf_precondition(h, r_ptr, w_ptr):
    _check(lib().lf_precondition(h, C.c_void_p(r_ptr), C.c_void_p(w_ptr)), "lf_precondition")


def lf_profile_enable(h, on):
    _check(lib().lf_profile_enable(h, C.c_int32(1 if on else 0)), "lf_profile_enable")


def lf_profile_read(h, n=16):
    ms = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int64)
    _check(lib().lf_profile_read(h, C.c_int32(n), C.c_void_p(ms.ctypes.data),
                                 C.c_void_p(cnt.ctypes.data)), "lf_profile_read")
    return ms, cnt


def lf_group_workspace_bytes(max_members):
    return int(lib().lf_group_workspace_bytes(C.c_int32(max_members)))


def lf_group_create(max_members, iters_per_block, ws_ptr, ws_bytes, stream):
    h = C.c_void_p()
    _check(lib().lf_group_create(C.c_int32(max_members), C.c_int32(iters_per_block), C.c_void_p(ws_ptr),
                                 C.c_size_t(ws_bytes), C.c_void_p(stream), C.byref(h)), "lf_group_create")
    return h


def lf_group_destroy(h):
    _check(lib().lf_group_destroy(h), "lf_group_destroy")


def lf_group_add(h, problem_h, n_steps, T0_ptr, snapshots_ptr, stats_array):
    _check(lib().lf_group_add(h, problem_h, C.c_int32(n_steps), C.c_void_p(T0_ptr or None),
                              C.c_void_p(snapshots_ptr or None),
                              C.cast(stats_array, C.c_void_p) if stats_array is not None else None),
           "lf_group_add")


def lf_group_poll(h, max_finished=64):
    out = (C.c_void_p * max(max_finished, 1))()
    nf, na = C.c_int32(0), C.c_int32(0)
    _check(lib().lf_group_poll(h, out, C.c_int32(max_finished), C.byref(nf), C.byref(na)), "lf_group_poll")
    return [out[i] for i in range(nf.value)], na.value


def lf_batch_workspace_bytes(max_tasks, max_steps):
    return int(lib().lf_batch_workspace_bytes(C.c_int32(max_tasks), C.c_int32(max_steps)))


def lf_batch_create(max_tasks, max_steps, ws_ptr, ws_bytes, stream):
    h = C.c_void_p()
    _check(lib().lf_batch_create(C.c_int32(max_tasks), C.c_int32(max_steps), C.c_void_p(ws_ptr),
                                 C.c_size_t(ws_bytes), C.c_void_p(stream), C.byref(h)),
           "lf_batch_create")
    return h


def lf_batch_destroy(h):
    _check(lib().lf_batch_destroy(h), "lf_batch_destroy")


def lf_batch_launch(h, problem_handles, snapshot_ptrs, n_steps, block_threads, n_workgroups=0):
    n = len(problem_handles)
    arr = (C.c_void_p * n)(*[ph.value for ph in problem_handles])
    snaps = None
    if snapshot_ptrs is not None:
        snaps = (C.c_void_p * n)(*[int(p) if p else None for p in snapshot_ptrs])
    _check(lib().lf_batch_launch(h, C.c_int32(n), arr, snaps, C.c_int32(n_steps),
                                 C.c_int32(block_threads), C.c_int32(n_workgroups)),
           "lf_batch_launch")


def lf_batch_poll(h):
    f = C.c_int32(0)
    _check(lib().lf_batch_poll(h, C.byref(f)), "lf_batch_poll")
    return bool(f.value)


def lf_batch_wait(h):
    _check(lib().lf_batch_wait(h), "lf_batch_wait")


def lf_batch_stats(h, n, n_steps):
    st = (lf_solve_stats * max(n * n_steps, 1))()
    ms = C.c_double(0.0)
    _check(lib().lf_batch_stats(h, st, C.byref(ms)), "lf_batch_stats")
    return [[st[i * n_steps + k].as_dict() for k in range(n_steps)] for i in range(n)], ms.value


# --------------------------------------------------------------------------
# convenience handles holding their torch workspaces
# --------------------------------------------------------------------------
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("lapfoam needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Mesh:
    """Device copy of a mesh (OpenFOAM face addressing) in a torch workspace.

    `m` has the fields of lf_mesh_desc as numpy arrays: n_cells, n_faces,
    owner, neighbour, cell_volume, cell_centre [N,3], face_area [F,3],
    patch_start, bface_cell, bface_area [B,3], bface_centre [B,3], and
    face_centre [F,3] when `gradient` (the mesh then serves `grad`).
    `non_orthogonal` accepts skewed faces; problems on such a mesh (created
    with `gradient`) apply the Laplacian's explicit non-orthogonal
    correction every step.
    """

    def __init__(self, m, stream=None, gradient=False, non_orthogonal=False):
        torch = _torch()
        self._keep = dict(
            owner=np.ascontiguousarray(m.owner, dtype=np.int32),
            neighbour=np.ascontiguousarray(m.neighbour, dtype=np.int32),
            cell_volume=np.ascontiguousarray(m.cell_volume, dtype=np.float64),
            cell_centre=np.ascontiguousarray(m.cell_centre, dtype=np.float64),
            face_area=np.ascontiguousarray(m.face_area, dtype=np.float64),
            patch_start=np.ascontiguousarray(m.patch_start, dtype=np.int32),
            bface_cell=np.ascontiguousarray(m.bface_cell, dtype=np.int32),
            bface_area=np.ascontiguousarray(m.bface_area, dtype=np.float64),
            bface_centre=np.ascontiguousarray(m.bface_centre, dtype=np.float64))
        if gradient:
            self._keep["face_centre"] = np.ascontiguousarray(m.face_centre, dtype=np.float64)
        k = self._keep
        self.n_cells = int(m.n_cells)
        self.n_faces = int(m.n_faces)
        self.n_patches = int(k["patch_start"].size - 1)
        self.n_bfaces = int(k["patch_start"][-1])
        d = lf_mesh_desc()
        d.n_cells, d.n_faces, d.n_patches = self.n_cells, self.n_faces, self.n_patches
        for name in ("owner", "neighbour", "cell_volume", "cell_centre", "face_area",
                     "patch_start", "bface_cell", "bface_area", "bface_centre"):
            setattr(d, name, k[name].ctypes.data)
        d.face_centre = k["face_centre"].ctypes.data if gradient else None
        d.flags = LF_MESH_NON_ORTHOGONAL if non_orthogonal else 0
        self.has_gradient = bool(gradient)
        self.desc = d
        self.ws_bytes = lf_mesh_workspace_bytes(d)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        assert self.ws.data_ptr() % 256 == 0
        self.stream = _stream_ptr(stream)
        self.h = lf_mesh_create(d, self.ws.data_ptr(), self.ws_bytes, self.stream)
        self.n_bands, self.band_offsets = lf_mesh_bands(self.h)
        del self._keep   # host arrays were read during the call only

    def cell_order(self):
        """(reordered, order): whether the solver keeps the cells in Morton order
        of their centres, and the mesh cell of each solver row."""
        return lf_mesh_cell_order(self.h, self.n_cells)

    def grad(self, T, Tb, snb=None, with_boundary=True):
        """Gauss gradient of the cell field T (device float64 tensor [N], mesh
        order) with boundary values Tb [B] and, for the boundary gradient,
        their normal gradients snb [B].  Returns (grad [N,3], bgrad [B,3] or
        None) as new device tensors, ordered on the mesh's stream."""
        torch = _torch()
        N, B = self.n_cells, self.n_bfaces
        for name, t, n in (("T", T, N), ("Tb", Tb, B)) + ((("snb", snb, B),) if with_boundary else ()):
            if t is None or t.dtype != torch.float64 or not t.is_cuda or t.numel() != n \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of {n} values")
        g = torch.empty((N, 3), dtype=torch.float64, device=T.device)
        bg = torch.empty((max(B, 1), 3), dtype=torch.float64, device=T.device) if with_boundary else None
        lf_grad(self.h, T.data_ptr(), Tb.data_ptr() if B else 0,
                snb.data_ptr() if (with_boundary and B) else 0, g.data_ptr(),
                bg.data_ptr() if with_boundary else 0)
        return g, (bg[:B] if with_boundary else None)

    def addressing(self):
        N, F, B = self.n_cells, self.n_faces, self.n_bfaces
        out = dict(owner_start=np.empty(N + 1, np.int32), losort=np.empty(max(F, 1), np.int32),
                   losort_start=np.empty(N + 1, np.int32), bface_start=np.empty(N + 1, np.int32),
                   bface_list=np.empty(max(B, 1), np.int32))
        lf_mesh_get_addressing(self.h, **out)
        out["losort"] = out["losort"][:F]
        out["bface_list"] = out["bface_list"][:B]
        return out

    def close(self):
        if getattr(self, "h", None):
            lf_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(tol=1e-9, rel_tol=0.0, max_iter=1000, min_iter=0, precond=LF_PC_DIAGONAL,
              precision=LF_PREC_FP64, iters_per_check=0, use_graph=1, inner_tol=0.0, max_outer=0,
              layout=LF_LAYOUT_AUTO, amul_walk=LF_WALK_AUTO, inner_restart=0, n_nonorth_corr=0):
    o = lf_default_opts()
    o.tol, o.rel_tol, o.max_iter, o.min_iter = tol, rel_tol, max_iter, min_iter
    o.precond, o.precision, o.iters_per_check, o.use_graph = precond, precision, iters_per_check, use_graph
    o.inner_tol, o.max_outer, o.layout, o.amul_walk = inner_tol, max_outer, layout, amul_walk
    o.inner_restart = inner_restart
    o.n_nonorth_corr = n_nonorth_corr
    return o


class Problem:
    """Mesh + boundary conditions + DT + dt + solver options, with field T."""

    def __init__(self, mesh, bcs, DT, dt, opts=None, stream=None):
        torch = _torch()
        self.mesh = mesh
        self.opts = opts if opts is not None else make_opts()
        arr = (lf_patch_bc * max(len(bcs), 1))()
        for i, (t, v) in enumerate(bcs):
            arr[i].type, arr[i].value = int(t), float(v)
        self.ws_bytes = lf_problem_workspace_bytes(mesh.h, self.opts)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        assert self.ws.data_ptr() % 256 == 0
        self.stream = _stream_ptr(stream) if stream is not None else mesh.stream
        self.h = lf_problem_create(mesh.h, arr, DT, dt, self.opts, self.ws.data_ptr(),
                                   self.ws_bytes, self.stream)
        self._async_steps, self._async_snap = 0, None     # lf_step_begin's run

    def grad(self, with_boundary=True):
        """Gauss gradient of the current T with the problem's boundary
        conditions: (grad [N,3], bgrad [B,3] or None), new device tensors in
        the mesh's order, ordered on the problem's stream."""
        torch = _torch()
        N, B = self.mesh.n_cells, self.mesh.n_bfaces
        g = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        bg = torch.empty((max(B, 1), 3), dtype=torch.float64, device="cuda") if with_boundary else None
        lf_problem_grad(self.h, g.data_ptr(), bg.data_ptr() if with_boundary else 0)
        return g, (bg[:B] if with_boundary else None)

    def layout(self):
        """LF_LAYOUT_ROWS or LF_LAYOUT_BANDS."""
        return lf_problem_layout(self.h)

    def amul_walk(self):
        """True if the FP64 matrix-vector product runs as a walk (row or block)
        or, with DIC on the two-colour layout, with two pairs per lane."""
        return bool(lf_problem_amul_walk(self.h))

    def amul_form(self):
        """0 one row per thread, 1 the row walk, 2 the block walk of a box,
        3 DIC's kernels on the two-colour layout with two red-black pairs per lane,
        4 the block walk with the FP64 diagonal solve on the Jacobi-scaled matrix."""
        return lf_problem_amul_walk(self.h)

    def reset(self, bcs, DT, dt):
        """New boundary conditions, DT and dt for the same mesh and workspace."""
        arr = (lf_patch_bc * max(len(bcs), 1))()
        for i, (t, v) in enumerate(bcs):
            arr[i].type, arr[i].value = int(t), float(v)
        lf_problem_reset(self.h, arr, DT, dt)

    def set_T(self, T):
        if hasattr(T, "data_ptr"):
            lf_set_T(self.h, T.data_ptr(), 1)
        else:
            a = np.ascontiguousarray(T, dtype=np.float64)
            lf_set_T(self.h, a.ctypes.data, 0)

    def get_T(self, out=None):
        if out is not None and hasattr(out, "data_ptr"):
            lf_get_T(self.h, out.data_ptr(), 1)
            return out
        a = np.empty(self.mesh.n_cells, np.float64)
        lf_get_T(self.h, a.ctypes.data, 0)
        return a

    def boundary_T(self):
        """Field values on the boundary faces (host array, boundary-face order)."""
        a = np.empty(max(self.mesh.n_bfaces, 1), np.float64)
        lf_get_boundary_T(self.h, a.ctypes.data, 0)
        return a[: self.mesh.n_bfaces]

    def step(self, n_steps=1, check=True):
        stats = (lf_solve_stats * max(n_steps, 1))()
        status = lf_step(self.h, n_steps, stats)
        if check:
            _check(status, "lf_step")
        return [s.as_dict() for s in stats[:n_steps]], status

    def step_begin(self, n_steps, snapshots=None):
        """Start n_steps time steps without waiting; snapshots: a device float64
        tensor of n_steps * n_cells values (mesh cell order) that receives T
        after each step, or None."""
        if snapshots is not None:
            assert snapshots.dtype.is_floating_point and snapshots.element_size() == 8
            assert snapshots.is_cuda and snapshots.is_contiguous()
            assert snapshots.numel() >= n_steps * self.mesh.n_cells
        self._async_steps = int(n_steps)
        self._async_snap = snapshots     # kept alive while the run may write it
        lf_step_begin(self.h, n_steps, snapshots.data_ptr() if snapshots is not None else None)

    def step_poll(self):
        """(steps_done, finished, stats of the finished steps, status), without waiting."""
        out = lf_step_poll(self.h, self._async_steps)
        if out[1]:
            self._async_snap = None
        return out

    def assemble(self):
        lf_assemble(self.h)

    def matrix(self):
        N, F, B = self.mesh.n_cells, self.mesh.n_faces, self.mesh.n_bfaces
        out = dict(diag=np.empty(N), upper=np.empty(max(F, 1)), source=np.empty(N),
                   diag_b=np.empty(N), source_b=np.empty(N), int_coeff=np.empty(max(B, 1)),
                   bou_coeff=np.empty(max(B, 1)))
        lf_get_matrix(self.h, **out)
        out["upper"] = out["upper"][:F]
        out["int_coeff"] = out["int_coeff"][:B]
        out["bou_coeff"] = out["bou_coeff"][:B]
        return out

    def amul(self, x, y):
        lf_amul(self.h, x.data_ptr(), y.data_ptr())

    def amul_inner(self, x, y):
        """y = A32 x, the mixed form's inner FP32 product (device float32 tensors,
        solver row order)."""
        lf_amul_inner(self.h, x.data_ptr(), y.data_ptr())

    def precondition(self, r, w):
        """w = M r with the problem's preconditioner (device float64 tensors)."""
        lf_precondition(self.h, r.data_ptr(), w.data_ptr())

    def profile(self, on=True):
        lf_profile_enable(self.h, on)

    def profile_read(self):
        ms, cnt = lf_profile_read(self.h, len(KERNEL_CLASSES))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(KERNEL_CLASSES)
                if cnt[i] > 0}

    def close(self):
        if getattr(self, "h", None):
            lf_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Problems stepped together: their inner FP32 iterations share launches
    (lf_group_*).  add() starts a member's run; poll() advances every member
    without waiting and returns [(problem, stats list)] of the finished runs."""

    def __init__(self, max_members, iters_per_block=0, stream=None):
        torch = _torch()
        self.max_members = max_members
        self.ws_bytes = lf_group_workspace_bytes(max_members)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream_obj = stream
        self.stream = _stream_ptr(stream)
        self.h = lf_group_create(max_members, iters_per_block, self.ws.data_ptr(), self.ws_bytes, self.stream)
        self._runs = {}            # problem handle value -> (problem, stats array, snapshots)

    def add(self, problem, n_steps, snapshots=None, T0=None):
        """Start problem's run of n_steps steps from T0 (device float64 tensor
        in mesh order, kept alive here until the run finishes) or its current T."""
        stats = (lf_solve_stats * n_steps)()
        lf_group_add(self.h, problem.h, n_steps, T0.data_ptr() if T0 is not None else 0,
                     snapshots.data_ptr() if snapshots is not None else 0, stats)
        self._runs[problem.h.value] = (problem, stats, snapshots, T0)

    def poll(self):
        handles, active = lf_group_poll(self.h, self.max_members)
        done = []
        for hv in handles:
            problem, stats, _, _ = self._runs.pop(hv)
            done.append((problem, [s.as_dict() for s in stats]))
        self.active = active
        return done

    def close(self):
        if getattr(self, "h", None):
            lf_group_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Persistent batched solver launches (one workgroup per problem at a time)."""

    def __init__(self, max_tasks, max_steps, stream=None):
        torch = _torch()
        self.max_tasks, self.max_steps = max_tasks, max_steps
        self.ws_bytes = lf_batch_workspace_bytes(max_tasks, max_steps)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream_obj = stream
        self.stream = _stream_ptr(stream)
        self.h = lf_batch_create(max_tasks, max_steps, self.ws.data_ptr(), self.ws_bytes, self.stream)
        self._n = 0
        self._steps = 0

    def launch(self, problems, n_steps, block_threads=512, n_workgroups=0, snapshots=None):
        ptrs = None if snapshots is None else [s.data_ptr() if s is not None else 0 for s in snapshots]
        lf_batch_launch(self.h, [p.h for p in problems], ptrs, n_steps, block_threads, n_workgroups)
        self._n, self._steps = len(problems), n_steps

    def poll(self):
        return lf_batch_poll(self.h)

    def wait(self):
        lf_batch_wait(self.h)

    def stats(self):
        return lf_batch_stats(self.h, self._n, self._steps)

    def close(self):
        if getattr(self, "h", None):
            lf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

