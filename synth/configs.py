"""The five workloads the path is measured and checked on, as seeded recipes.

plain_32      32^3 uniform unit cube, DT=1e-3, dt=5e-3, 20 steps, diagonal PCG
graded_256    256^3 box graded in z (expansion ratio 10), DT=1e-3, dt=1e-3, 50 steps,
              diagonal PCG, and red-black DIC on the red-black renumbered mesh
permuted_192  192^3 graded box, cells randomly relabelled (seed 1), DT=5e-4,
              dt=1e-3, 30 steps, diagonal PCG
mixed_256     graded_256's problem solved by FP32-inner / FP64-outer refinement
stream_512    512 requests, cube side log-uniform in [16, 96], DT log-uniform in
              [1e-4, 1e-2], dt=1e-3, 10 steps each, Poisson arrivals

All: fixedValue 273 K at x=0 and 573 K at x=1, zeroGradient elsewhere;
T0 ~ U[273, 573) from seed 20250724; normalised-residual tolerance 1e-9,
relative tolerance 0, at most 1000 iterations.
"""
import math
from dataclasses import dataclass
from typing import List

import numpy as np

from .mesh import (box_mesh, renumber, random_permutation, red_black_numbering,
                   initial_field, fixed_x_bcs)
from .rng import uniform01

T0_SEED = 20250724
PERM_SEED = 1
STREAM_SEED = 7

CONFIGS = {
    "plain_32": dict(n=32, z_ratio=1.0, DT=1e-3, dt=5e-3, steps=20, numbering="natural",
                     precond="diagonal"),
    "graded_256": dict(n=256, z_ratio=10.0, DT=1e-3, dt=1e-3, steps=50, numbering="natural",
                       precond="diagonal"),
    "graded_256_dic": dict(n=256, z_ratio=10.0, DT=1e-3, dt=1e-3, steps=50,
                           numbering="red_black", precond="dic"),
    "permuted_192": dict(n=192, z_ratio=10.0, DT=5e-4, dt=1e-3, steps=30, numbering="random",
                         precond="diagonal"),
    "mixed_256": dict(n=256, z_ratio=10.0, DT=1e-3, dt=1e-3, steps=50, numbering="natural",
                      precond="diagonal", precision="mixed"),
}
TOL = 1e-9
REL_TOL = 0.0
MAX_ITER = 1000


@dataclass
class Problem:
    name: str
    mesh: object
    bcs: list
    DT: float
    dt: float
    steps: int
    T0: np.ndarray
    precond: str
    precision: str
    n_red: int = 0


def build_config(name: str, n: int = None, steps: int = None) -> Problem:
    """Build a config's mesh and initial field; `n` overrides the cube side."""
    cfg = CONFIGS[name]
    side = cfg["n"] if n is None else n
    mesh = box_mesh(side, side, side, z_ratio=cfg["z_ratio"])
    new_of_old = None
    n_red = 0
    if cfg["numbering"] == "random":
        new_of_old = random_permutation(mesh.n_cells, PERM_SEED)
    elif cfg["numbering"] == "red_black":
        new_of_old, n_red = red_black_numbering(mesh)
    if new_of_old is not None:
        mesh = renumber(mesh, new_of_old)
    T0 = initial_field(mesh.n_cells, T0_SEED, new_of_old=new_of_old)
    return Problem(name=name, mesh=mesh, bcs=fixed_x_bcs(), DT=cfg["DT"], dt=cfg["dt"],
                   steps=cfg["steps"] if steps is None else steps, T0=T0,
                   precond=cfg["precond"], precision=cfg.get("precision", "fp64"),
                   n_red=n_red)


@dataclass
class Request:
    rid: int
    arrival: float      # seconds after stream start
    n: int              # cube side
    DT: float
    dt: float
    steps: int
    seed: int           # T0 seed


def request_stream(n_requests: int = 512, rate: float = 1.0, seed: int = STREAM_SEED,
                   n_lo: int = 16, n_hi: int = 96, dt_lo: float = 1e-4, dt_hi: float = 1e-2,
                   dt: float = 1e-3, steps: int = 10) -> List[Request]:
    """Poisson arrivals (rate per second); side and DT log-uniform.

    Independent SplitMix64 streams of one seed: draws [0,R) inter-arrival,
    [R,2R) side, [2R,3R) DT.  Request r's T0 uses seed T0_SEED + r.
    """
    R = n_requests
    u = uniform01(seed, 3 * R)
    inter = -np.log1p(-u[:R]) / rate
    arrival = np.cumsum(inter) - inter[0]
    side = np.clip(np.rint(np.exp(math.log(n_lo) + u[R:2 * R] * (math.log(n_hi) - math.log(n_lo)))),
                   n_lo, n_hi).astype(int)
    DTs = np.exp(math.log(dt_lo) + u[2 * R:] * (math.log(dt_hi) - math.log(dt_lo)))
    return [Request(rid=r, arrival=float(arrival[r]), n=int(side[r]), DT=float(DTs[r]), dt=dt,
                    steps=steps, seed=T0_SEED + r) for r in range(R)]
