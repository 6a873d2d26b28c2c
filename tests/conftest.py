import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def small_workload():
    """hybrid10k recipe at n = 2000 with 30 queries per fraction (oracle-only tests)."""
    from synth import workloads as w
    spec = w.scaled(w.SPECS["hybrid10k"], n=2000, nq=30)
    return w.make(spec, base_seed=11)


@pytest.fixture(scope="session")
def small_index(small_workload):
    from oracle import hsig
    W = small_workload
    s = W.spec
    return hsig.Index.build(W.base, W.attr, W.level_u, s.S, s.M, s.ef_cons, seed=11)
