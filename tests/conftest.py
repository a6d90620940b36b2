import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def golden_dir():
    return GOLDEN


def read_pool(name):
    """Rows of a pool golden file written by tests/golden/make_*.py: {index:
    dict(words, states, transitions, deadlocks, dead_digest, levels)}."""
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x) for x in line.split()]
        rows[v[0]] = {"words": v[1], "states": v[2], "transitions": v[3], "deadlocks": v[4],
                      "dead_digest": (v[5], v[6]), "levels": v[7:]}
    return rows
