import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


_CACHE = {}


def cached_workload(name, n, nq, L=None, ncomp=None, **kw):
    """Seeded small workload + trained index, cached per test session."""
    from workloads import make_workload, scaled, train_index
    key = (name, n, nq, L, ncomp, tuple(sorted(kw.items())))
    if key not in _CACHE:
        cfg = scaled(name, n=n, nq=nq, L=L, ncomp=ncomp, **kw) if name != "c1" or n != 10_000 \
            else __import__("workloads").CONFIGS["c1"]
        X, Q, nprobe = make_workload(cfg)
        index = train_index(X, cfg)
        _CACHE[key] = (cfg, X, Q, nprobe, index)
    return _CACHE[key]


@pytest.fixture(scope="session")
def c1_workload():
    return cached_workload("c1", 10_000, 100)


def make_rng(*seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2511, 3298, 99, *seed])))
