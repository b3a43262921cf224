"""The pins catch plausible slips in the oracle (no GPU).

Each case plants one mistake in a copy of the oracle's source (a text
substitution), builds it with the oracle's own flags into a temporary
directory, and runs the face-factor and weight pins against it: at least one
pin must fail.  The unmodified source passes them all (test_oracle_geometry).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import build as obuild
from oracle import oracle as O
from tests import test_oracle_amg as M
from tests import test_oracle_geometry as G

SRC = os.path.join(os.path.dirname(obuild.__file__), "lforacle.c")

# (name, text in the oracle's source, its replacement); the face-factor pins
MUTANTS = [
    ("delta_f over |d|", "delta[f] = 1.0 / (nd > lim ? nd : lim);", "delta[f] = 1.0 / dmag;"),
    ("delta_f without limiter", "delta[f] = 1.0 / (nd > lim ? nd : lim);", "delta[f] = 1.0 / nd;"),
    ("delta_f limiter on 0.5|d|", "double lim = 0.05 * dmag;", "double lim = 0.5 * dmag;"),
    ("delta_b over |C_b - C_P|", "bdelta[b] = 1.0 / nd;",
     "bdelta[b] = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);"),
    ("weights without fallback", "w[f] = fabs(den) > LFO_ROOTVSMALL ? sfd_nei / den : 0.5;",
     "w[f] = sfd_nei / den;"),
    ("fallback at VSMALL", "#define LFO_ROOTVSMALL 1.0e-150", "#define LFO_ROOTVSMALL 1.0e-300"),
    ("weights swapped", "w[f] = fabs(den) > LFO_ROOTVSMALL ? sfd_nei / den : 0.5;",
     "w[f] = fabs(den) > LFO_ROOTVSMALL ? sfd_own / den : 0.5;"),
    ("boundary coefficient without delta_b", "double lap_bc = -(gamma_b * (bdelta[b] * patch_value[p]));",
     "double lap_bc = -(gamma_b * patch_value[p]);"),
]

# the same for the multigrid pins
AMG_MUTANTS = [
    ("restriction averages", "bc[L->agg[c]] += y[c];", "bc[L->agg[c]] += 0.125 * y[c];"),
    ("prolongation dropped", "x[c] += xc[L->agg[c]];", "x[c] += 0.0 * xc[L->agg[c]];"),
    ("internal face counted once", "cdiag[I] += 2.0 * upper[f];", "cdiag[I] += upper[f];"),
    ("coarse face keeps one fine face", "cupper[k] += upper[pairs[i].f];", "cupper[k] = upper[pairs[i].f];"),
    ("Jacobi without the diagonal", "x[c] = x[c] + omega * ((b[c] - y[c]) / L->diag[c]);",
     "x[c] = x[c] + omega * (b[c] - y[c]);"),
    ("no smoothing after the correction",
     "x[c] += xc[L->agg[c]];\n        for (int32_t s = 0; s < h->nu; ++s)",
     "x[c] += xc[L->agg[c]];\n        for (int32_t s = 0; s < 0; ++s)"),
    ("coarse right side from b, not the residual", "bc[L->agg[c]] += y[c];", "bc[L->agg[c]] += b[c];"),
]


def _build(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *obuild.CFLAGS, "-o", str(lib), str(path), "-lm"], check=True)
    return ctypes.CDLL(str(lib))


def _failing_pins(tmp_path, old, new, pins):
    O.lib()
    mutant = _build(tmp_path, old, new)
    saved = O._lib
    failed = []
    try:
        O._lib = mutant
        for pin in pins:
            try:
                pin(O)
            except (AssertionError, np.linalg.LinAlgError):
                failed.append(pin.__name__)
    finally:
        O._lib = saved
    return failed


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_slip_fails_a_pin(tmp_path, name, old, new):
    assert _failing_pins(tmp_path, old, new, G.PINS), f"no pin caught the planted slip '{name}'"


@pytest.mark.parametrize("name,old,new", AMG_MUTANTS, ids=[m[0] for m in AMG_MUTANTS])
def test_planted_multigrid_slip_fails_a_pin(tmp_path, name, old, new):
    assert _failing_pins(tmp_path, old, new, M.PINS), f"no pin caught the planted slip '{name}'"
