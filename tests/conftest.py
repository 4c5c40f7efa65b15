"""Shared fixtures.  Tests marked ``gpu`` need an MI355X and the built HIP
library; everything else runs on the CPU."""

import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


_cache = {}


@pytest.fixture(scope="session")
def oracle_levels():
    """Oracle levels of the plain FP64 workload (unit icosphere s=1..3, k=1,
    d=e_z, p=e_x, radial field), built once per session."""
    import workloads
    from oracle import uq

    def get(s: int, k: float = 1.0, field_kind: str = "radial"):
        key = (s, k, field_kind)
        if key not in _cache:
            zkey = (s, k, "radial")
            Z = _cache[zkey].Z if zkey in _cache else None
            _cache[key] = uq.make_level(*workloads.icosphere(s), k, field_kind=field_kind, Z=Z)
        return _cache[key]

    return get
