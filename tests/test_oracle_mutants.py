"""The pins catch plausible slips in the oracle (no GPU).

Each case plants one mistake in a copy of the oracle's source (a text
substitution), builds it with the oracle's own flags into a temporary
directory, and runs the face-factor and weight pins against it: at least one
pin must fail.  The unmodified source passes them all (test_oracle_geometry).
"""
import ctypes
import os
import subprocess

import pytest

from oracle import build as obuild
from oracle import oracle as O
from tests import test_oracle_geometry as G

SRC = os.path.join(os.path.dirname(obuild.__file__), "lforacle.c")

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


def _build(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *obuild.CFLAGS, "-o", str(lib), str(path), "-lm"], check=True)
    return ctypes.CDLL(str(lib))


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_slip_fails_a_pin(tmp_path, name, old, new):
    O.lib()
    mutant = _build(tmp_path, old, new)
    saved = O._lib
    failed = []
    try:
        O._lib = mutant
        for pin in G.PINS:
            try:
                pin(O)
            except AssertionError:
                failed.append(pin.__name__)
    finally:
        O._lib = saved
    assert failed, f"no pin caught the planted slip '{name}'"
