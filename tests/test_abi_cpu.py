"""The C-ABI library loads on a machine without a GPU, exports every function
the header declares, and its ctypes structures match the C layout."""
import os
import re
import subprocess
import ctypes as C

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lapfoam.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lf_mesh_create", "lf_problem_create", "lf_step", "lf_amul", "lf_set_T",
                 "lf_get_T", "lf_mesh_workspace_bytes", "lf_problem_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2507_18268_amd import lapfoam as L
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    nm = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r" T (lf_[A-Za-z_0-9]+)", nm))
    assert set(declared_functions()) <= exported


def test_binding_covers_every_declared_symbol():
    from paper_2507_18268_amd import lapfoam as L
    assert set(declared_functions()) <= set(L._SIGS)


def test_struct_layouts_match_c(tmp_path):
    from paper_2507_18268_amd import lapfoam as L
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "lapfoam.h"
#define P(T, f) printf(#T "." #f " %zu\\n", offsetof(T, f));
int main(void) {
  printf("lf_mesh_desc %zu\\n", sizeof(lf_mesh_desc));
  printf("lf_patch_bc %zu\\n", sizeof(lf_patch_bc));
  printf("lf_solver_opts %zu\\n", sizeof(lf_solver_opts));
  printf("lf_solve_stats %zu\\n", sizeof(lf_solve_stats));
  P(lf_mesh_desc, bface_centre) P(lf_solver_opts, layout) P(lf_solver_opts, inner_tol)
  P(lf_solve_stats, solve_ms) P(lf_patch_bc, value)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True,
                                                              text=True).stdout.split("\n") if line)
    assert int(out["lf_mesh_desc"]) == C.sizeof(L.lf_mesh_desc)
    assert int(out["lf_patch_bc"]) == C.sizeof(L.lf_patch_bc)
    assert int(out["lf_solver_opts"]) == C.sizeof(L.lf_solver_opts)
    assert int(out["lf_solve_stats"]) == C.sizeof(L.lf_solve_stats)
    assert int(out["lf_mesh_desc.bface_centre"]) == L.lf_mesh_desc.bface_centre.offset
    assert int(out["lf_solver_opts.layout"]) == L.lf_solver_opts.layout.offset
    assert int(out["lf_solver_opts.inner_tol"]) == L.lf_solver_opts.inner_tol.offset
    assert int(out["lf_solve_stats.solve_ms"]) == L.lf_solve_stats.solve_ms.offset
    assert int(out["lf_patch_bc.value"]) == L.lf_patch_bc.value.offset


def test_host_only_entry_points_without_gpu():
    """Calls that need no device: defaults, workspace sizing, error paths."""
    from paper_2507_18268_amd import lapfoam as L
    import numpy as np
    import synth
    o = L.lf_default_opts()
    assert o.tol == 1e-9 and o.max_iter == 1000 and o.precond == L.LF_PC_DIAGONAL
    m = synth.box_mesh(3, 2, 2)
    d = L.lf_mesh_desc()
    arrs = dict(owner=m.owner, neighbour=m.neighbour, cell_volume=m.cell_volume,
                cell_centre=np.ascontiguousarray(m.cell_centre), face_area=m.face_area,
                patch_start=m.patch_start, bface_cell=m.bface_cell, bface_area=m.bface_area,
                bface_centre=m.bface_centre)
    d.n_cells, d.n_faces, d.n_patches = m.n_cells, m.n_faces, m.n_patches
    for k, v in arrs.items():
        setattr(d, k, v.ctypes.data)
    nbytes = L.lf_mesh_workspace_bytes(d)
    assert nbytes > 0 and nbytes % 256 == 0
    # a workspace that is too small is refused before any device call
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 16, 0)
    assert e.value.status == L.LF_ENOMEM
    # invalid mesh: owner >= neighbour
    bad = m.owner.copy()
    bad[0] = m.neighbour[0]
    d.owner = bad.ctypes.data
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, nbytes, 0)
    assert e.value.status == L.LF_EMESH
    assert "owner" in L.lf_last_error()


def _desc(L, m, keep):
    import numpy as np
    d = L.lf_mesh_desc()
    arrs = dict(owner=m["owner"], neighbour=m["neighbour"], cell_volume=m["cell_volume"],
                cell_centre=m["cell_centre"], face_area=m["face_area"], patch_start=m["patch_start"],
                bface_cell=m["bface_cell"], bface_area=m["bface_area"], bface_centre=m["bface_centre"])
    for k, v in arrs.items():
        v = np.ascontiguousarray(v)
        keep.append(v)
        setattr(d, k, v.ctypes.data)
    d.n_cells, d.n_faces, d.n_patches = m["n_cells"], m["owner"].size, m["patch_start"].size - 1
    return d


def _box_dict(m):
    return dict(owner=m.owner.astype("int32"), neighbour=m.neighbour.astype("int32"),
                cell_volume=m.cell_volume, cell_centre=m.cell_centre, face_area=m.face_area,
                patch_start=m.patch_start.astype("int32"), bface_cell=m.bface_cell.astype("int32"),
                bface_area=m.bface_area, bface_centre=m.bface_centre, n_cells=m.n_cells)


@pytest.mark.parametrize("defect", ["unsorted", "non_orthogonal", "inward_boundary", "bad_index",
                                    "zero_volume"])
def test_mesh_validation_rejects(defect):
    """Host validation (no device call is made before it fails)."""
    from paper_2507_18268_amd import lapfoam as L
    import synth
    m = _box_dict(synth.box_mesh(4, 3, 3))
    m = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in m.items()}
    if defect == "unsorted":
        m["owner"][[0, 1]] = m["owner"][[1, 0]]
        m["neighbour"][[0, 1]] = m["neighbour"][[1, 0]]
        m["face_area"][[0, 1]] = m["face_area"][[1, 0]]
    elif defect == "non_orthogonal":
        m["face_area"][5] = m["face_area"][5] + [0.0, 0.3 * abs(m["face_area"][5]).max(), 0.0]
    elif defect == "inward_boundary":
        m["bface_area"][2] = -m["bface_area"][2]
    elif defect == "bad_index":
        m["neighbour"][-1] = m["n_cells"]
    elif defect == "zero_volume":
        m["cell_volume"][7] = 0.0
    keep = []
    d = _desc(L, m, keep)
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 1 << 20, 0)
    assert e.value.status == L.LF_EMESH, L.lf_last_error()


def test_mesh_rows_longer_than_255_are_refused():
    """A cell with 256 faces exceeds the row layout's uint8 row length: LF_EMESH
    (and a zero workspace size), before any device call."""
    from paper_2507_18268_amd import lapfoam as L
    import numpy as np
    k = 256
    ang = np.linspace(0.0, np.pi, k + 2)[1:-1]
    dirs = np.stack([np.cos(ang), np.sin(ang), np.zeros(k)], axis=1)     # all distinct, in one half-plane
    centres = np.concatenate([np.zeros((1, 3)), dirs], axis=0)
    m = dict(owner=np.zeros(k, np.int32), neighbour=np.arange(1, k + 1, dtype=np.int32),
             cell_volume=np.full(k + 1, 1e-3), cell_centre=centres, face_area=0.01 * dirs,
             patch_start=np.zeros(1, np.int32), bface_cell=np.zeros(0, np.int32),
             bface_area=np.zeros((0, 3)), bface_centre=np.zeros((0, 3)), n_cells=k + 1)
    keep = []
    d = _desc(L, m, keep)
    assert L.lf_mesh_workspace_bytes(d) == 0
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 1 << 20, 0)
    assert e.value.status == L.LF_EMESH and "255" in L.lf_last_error()


def test_mesh_flags_on_host():
    """LF_MESH_NON_ORTHOGONAL lets a skewed box past validation (the call then
    stops at the missing workspace, before any device call); unknown flags are
    refused; face centres add the gradient's records to the workspace."""
    from paper_2507_18268_amd import lapfoam as L
    import numpy as np
    import synth
    mesh = synth.affine(synth.box_mesh(4, 3, 3), synth.SKEW)
    keep = []
    d = _desc(L, _box_dict(mesh), keep)
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 1 << 20, 0)
    assert e.value.status == L.LF_EMESH
    d.flags = L.LF_MESH_NON_ORTHOGONAL
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 1 << 20, 0)
    assert e.value.status == L.LF_ENOMEM, L.lf_last_error()
    d.flags = 4
    with pytest.raises(L.LapfoamError) as e:
        L.lf_mesh_create(d, 0, 1 << 20, 0)
    assert e.value.status == L.LF_EINVAL
    d.flags = L.LF_MESH_NON_ORTHOGONAL
    plain = L.lf_mesh_workspace_bytes(d)
    fc = np.ascontiguousarray(mesh.face_centre)
    d.face_centre = fc.ctypes.data
    with_grad = L.lf_mesh_workspace_bytes(d)
    assert with_grad >= plain + 32 * (mesh.n_faces + mesh.n_bfaces)
