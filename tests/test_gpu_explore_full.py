"""Parity of gx_explore on the large plain-path workload: 12 processes of 64
declared states (3-word vectors), 3,304,390,656 reachable states in a 192 GB
table, explored in the table configuration the benchmark times
(``workloads.LARGE_EXPLORE``).

The exact result comes from the oracle alone: ``oracle.explore_dense`` (the
same BFS over dense bitmaps, pinned in test_oracle_dense_cpu.py) computed the
state and transition counts, every level count, the deadlock count and an
order-independent digest of the reachable set, stored in
``tests/golden/large_random_l8.txt`` by ``tests/golden/make_large_random_l8.py``.
The GPU exploration must reproduce all of them, and the table must hold
exactly the reachable set: as many occupied slots as states, with the
oracle's digest (computed window by window over the raw table on the
device).  The same family at a size the hash-set oracle enumerates (4 live
states per process) is compared bit-exactly, sorted table dump included."""
import os

import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

from conftest import GOLDEN
from setdigest import table_digest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _golden():
    out = {}
    for line in open(os.path.join(GOLDEN, "large_random_l8.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, *v = line.split()
            out[k] = [int(x) for x in v]
    return out


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def test_same_family_at_oracle_size_bit_exact(dev):
    net = W.large_random_network(live=4)
    want = oracle.explore(net, want_visited=True)
    cfg = dict(W.LARGE_EXPLORE)
    with gx.Table(3, cfg.pop("bucket_words"), 2 * want.n_states, **cfg) as t:
        got = gx.explore(net, t)
        assert got.n_states == want.n_states == 248832
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)
        n, dig = table_digest(t, dev)
        assert (n, dig) == (want.n_states, oracle.digest(want.visited, 3))


def test_full_size_exact(dev):
    g = _golden()
    torch.cuda.empty_cache()  # room for the 192 GB table
    net = W.large_random_network()
    cfg = dict(W.LARGE_EXPLORE)
    with gx.Table(3, cfg.pop("bucket_words"), W.LARGE_TABLE_SLOTS, **cfg) as t:
        r = gx.explore(net, t)
        print(f"explored {r.n_states} states, {len(r.levels)} levels", flush=True)
        assert r.n_states == g["states"][0]
        assert r.levels.tolist() == g["level_counts"]
        assert r.n_transitions == g["transitions"][0]
        assert len(r.deadlocks) == g["deadlocks"][0]
        assert oracle.digest(r.deadlocks, 3) == tuple(g["dead_digest"])
        s = t.stats()
        assert s.stored == r.n_states and s.full == 0
        n, dig = table_digest(t, dev)
        assert n == g["states"][0]
        assert dig == tuple(g["digest"])
