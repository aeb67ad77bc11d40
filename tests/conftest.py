import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


def read_golden(name):
    """Parse a ``key value`` fixture file (comments start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(" ")
            out[key] = val.strip()
    return out


def parse_adj(spec, n):
    adj = [[] for _ in range(n)]
    for tok in spec.split():
        v, _, lst = tok.partition(":")
        adj[int(v)] = [int(x) for x in lst.split(",") if x != ""]
    return adj


def adj_to_csr(adj):
    import numpy as np
    n = len(adj)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i, a in enumerate(adj):
        cols.extend(a)
        row_ptr[i + 1] = len(cols)
    return row_ptr, np.array(cols, dtype=np.int32)


@pytest.fixture(scope="session")
def golden():
    return read_golden
