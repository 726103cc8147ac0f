import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU case")


_cache = {}


def connectome(name, **kw):
    """Seeded synthetic problem, cached per test session."""
    import synth
    key = (name, tuple(sorted(kw.items())))
    if key not in _cache:
        _cache[key] = synth.make(name, **kw)
    return _cache[key]


@pytest.fixture(scope="session")
def tiny():
    return connectome("tiny")


def relerr(x, ref):
    """Normwise relative error ||x - ref||_2 / ||ref||_2 (ref = 0 -> ||x||)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(x - ref)
    n = np.linalg.norm(ref)
    return float(d / n) if n > 0 else float(d)
