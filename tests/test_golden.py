"""Values the paper prints, held against the oracle (fixtures under
tests/golden/, each citing its passage)."""

import os

from oracle.rwg import build_rwg
from workloads import flat_plate

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture(name):
    vals = {}
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = int(v)
    return vals


def test_plate_unknown_count():
    """Sec. V.C.2: the 20-wavelength plate at lambda/10 has 119,600 unknowns."""
    g = _fixture("plate_20lambda_unknowns.txt")
    xyz, tri = flat_plate(float(g["side_wavelengths"]), g["cells_per_side"])
    assert len(tri) == 2 * g["cells_per_side"] ** 2
    rwg = build_rwg(xyz, tri, allow_open=True)
    assert rwg["N"] == g["unknowns"]
