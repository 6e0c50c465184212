import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


_CACHE = {}


def cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def c0_workload():
    from workloads import workload
    return cached("c0w", lambda: workload("sphere_s3_200MHz"))


@pytest.fixture(scope="session")
def c0_hmatrix(c0_workload):
    from oracle.hmatrix import build_hmatrix
    w = c0_workload
    return cached("c0H", lambda: build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"],
                                               w["aca_tol"], workers=min(8, os.cpu_count() or 1)))


@pytest.fixture(scope="session")
def c0_dense(c0_hmatrix):
    return cached("c0Z", lambda: c0_hmatrix.op.dense())


@pytest.fixture(scope="session")
def small_sphere():
    """icosphere subdiv 2 (480 unknowns) at 300 MHz, leaf <= 16: 56 groups."""
    from workloads import icosphere
    from oracle.hmatrix import build_hmatrix

    def make():
        xyz, tri = icosphere(2, 1.0)
        return build_hmatrix(xyz, tri, 300e6, 16, 1e-3, workers=min(8, os.cpu_count() or 1))
    return cached("smallH", make)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
