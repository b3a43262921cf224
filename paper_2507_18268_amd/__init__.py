"""MI355X (gfx950) laplacianFoam hot path: implicit-Euler assembly of
ddt(T) - laplacian(DT, T) into an LDU matrix and its PCG solve, as a C-ABI
HIP library (liblapfoam.so) with a thin ctypes binding."""
from . import lapfoam  # noqa: F401
