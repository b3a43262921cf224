"""Shared helpers of the GPU tests (they call the library through its C ABI)."""
import numpy as np
import pytest


def lapfoam():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a ROCm GPU")
    from paper_2507_18268_amd import lapfoam as L
    L.lib()
    return L


def run_gpu(L, mesh, bcs, DT, dt, T0, steps, keep_all=True, **opts):
    """Step on the GPU one step at a time; returns (T per step, stats per step)."""
    m = L.Mesh(mesh)
    P = L.Problem(m, bcs, DT, dt, L.make_opts(**opts))
    P.set_T(T0)
    Ts, stats = [], []
    if keep_all:
        for _ in range(steps):
            st, _ = P.step(1)
            stats += st
            Ts.append(P.get_T())
    else:
        st, _ = P.step(steps)
        stats += st
        Ts.append(P.get_T())
    P.close()
    m.close()
    return Ts, stats


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
