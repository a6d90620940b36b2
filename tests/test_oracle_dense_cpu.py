"""Pins of the oracle's dense-bitmap BFS (``oracle.explore_dense``) and of the
set digest used to compare reachable sets too large to list.

The dense BFS is what fixes the large plain-path workload exactly (3.3e9
states, ``tests/golden/large_random_l8.txt``), so it is pinned here against
what the paper and mathematics fix and against the two other oracle searches
(the hash-set BFS and the brute-force fixpoint), on the same network family
at sizes those finish in seconds."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

from setdigest import digest_words
from test_oracle_pins import DEGENERATE, _cycle_levels, _read_table, _tiny_random

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _same(a, d):
    """Hash-set or brute-force result ``a`` equals dense result ``d``."""
    assert d.n_states == a.n_states
    assert d.n_transitions == a.n_transitions
    assert d.levels.tolist() == a.levels.tolist()
    assert d.n_deadlocks == len(a.deadlocks)
    assert np.array_equal(d.deadlocks, a.deadlocks)
    assert np.array_equal(d.visited, a.visited)
    assert d.digest == oracle.digest(a.visited, d.words)
    assert d.dead_digest == oracle.digest(a.deadlocks, d.words)


@pytest.mark.parametrize("live", [3, 4])
def test_dense_equals_bfs_on_large_family(live):
    net = W.large_random_network(live=live)
    _same(oracle.explore(net, want_visited=True), oracle.explore_dense(net, want_visited=True))


@pytest.mark.parametrize("seed", range(30))
def test_dense_equals_bruteforce(seed):
    net = _tiny_random(seed)
    _same(oracle.bruteforce(net, want_visited=True), oracle.explore_dense(net, want_visited=True))


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_dense_does_not_depend_on_threads(threads):
    net = W.large_random_network(live=4)
    ref = oracle.explore_dense(net, threads=1)
    d = oracle.explore_dense(net, threads=threads)
    assert d.levels.tolist() == ref.levels.tolist()
    assert (d.n_transitions, d.digest, d.n_deadlocks) == (ref.n_transitions, ref.digest,
                                                         ref.n_deadlocks)


@pytest.mark.parametrize("sizes", [(8, 8, 8, 8), (3, 5, 7), (2,), (4, 1, 6), (16, 9)])
def test_dense_independent_cycles(sizes):
    d = oracle.explore_dense(W.independent_cycles(sizes))
    assert d.n_states == int(np.prod(sizes)) == d.index_space
    assert d.levels.tolist() == _cycle_levels(sizes).tolist()
    assert d.n_transitions == int(np.prod(sizes)) * len(sizes)
    assert d.n_deadlocks == 0


@pytest.mark.parametrize("n", range(2, 13))
def test_dense_token_ring(n):
    # printed in Table 1 (Sec. 5.2), closed form 2N * 3^(N-1)
    printed = dict(_read_table("token_ring_table1.txt"))
    d = oracle.explore_dense(W.token_ring(n))
    assert d.n_states == printed[n] == 2 * n * 3 ** (n - 1)
    assert d.n_deadlocks == 0


def test_dense_fig1_and_tiny():
    d = oracle.explore_dense(W.fig1_producer_consumers())
    assert (d.n_states, d.n_transitions) == (8, 24)
    d = oracle.explore_dense(W.tiny_cycles())
    assert (d.n_states, d.n_transitions, len(d.levels)) == (4096, 16512, 21)


@pytest.mark.parametrize("P,k", [(2, 3), (4, 4), (6, 5)])
def test_dense_wide_rule(P, k):
    d = oracle.explore_dense(W.wide_rule(P, k), want_visited=True)
    assert d.n_states == 1 + k ** P
    assert d.levels.tolist() == [1, k ** P]
    assert d.n_deadlocks == k ** P


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_dense_degenerate(name):
    n, levels, trans, dead = DEGENERATE[name]
    d = oracle.explore_dense(W.degenerate_networks()[name])
    assert (d.n_states, d.levels.tolist(), d.n_transitions, d.n_deadlocks) == (n, levels, trans,
                                                                               dead)


def test_dense_deadlock_cap():
    d = oracle.explore_dense(W.wide_rule(4, 4), dead_cap=10)
    assert d.n_deadlocks == 256 and d.deadlocks is None
    full = oracle.explore_dense(W.wide_rule(4, 4))
    assert d.dead_digest == full.dead_digest == oracle.digest(full.deadlocks, full.words)


def test_dense_index_space_limit():
    with pytest.raises(OverflowError):
        oracle.explore_dense(W.large_random_network(live=4), max_index_space=1000)


def test_large_golden_file_is_consistent(golden_dir):
    g = {}
    for line in open(os.path.join(golden_dir, "large_random_l8.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, *v = line.split()
            g[k] = [int(x) for x in v]
    assert len(g["level_counts"]) == g["levels"][0] == 38
    assert sum(g["level_counts"]) == g["states"][0] == 3_304_390_656
    assert g["level_counts"][0] == 1
    # the index space is the product of the processes' locally reachable counts
    net = W.large_random_network(live=8)
    space = 1
    for p in range(net.n_procs):
        seen, todo = {int(net.initial[p])}, [int(net.initial[p])]
        while todo:
            s = todo.pop()
            for src, _, dst in net.trans[p].tolist():
                if src == s and dst not in seen:
                    seen.add(dst)
                    todo.append(dst)
        space *= len(seen)
    assert g["index_space"][0] == space


# ------------------------------------------------------------------ digest
@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_torch_digest_equals_oracle_digest(w):
    rng = np.random.default_rng(100 + w)
    st = rng.integers(0, 2**32 - 1, size=(5000, w), dtype=np.uint64).astype(np.uint32)
    st[:4] = [0x7FFFFFFF] * w  # a word equal to p reduces to 0
    st[4:8] = [0xFFFFFFFE] * w
    st[8:12] = 0
    x = torch.from_numpy(st.astype(np.int64))
    assert digest_words(x, w) == oracle.digest(st, w)


def test_digest_is_order_independent_and_sensitive():
    rng = np.random.default_rng(7)
    st = rng.integers(0, 2**31, size=(4000, 3), dtype=np.uint64).astype(np.uint32)
    d = oracle.digest(st, 3)
    assert oracle.digest(st[rng.permutation(4000)], 3) == d
    for i in range(20):  # any single changed word changes both sums
        bad = st.copy()
        bad[i * 37, i % 3] ^= np.uint32(1 << (i % 31))
        e = oracle.digest(bad, 3)
        assert e[0] != d[0] and e[1] != d[1]
    # a missing state and a duplicated one keep the count but change the digest
    bad = st.copy()
    bad[5] = bad[6]
    assert oracle.digest(bad, 3) != d


@pytest.mark.parametrize("name", ["batch_1024_s11.txt", "served_pool.txt"])
def test_pool_golden_files_are_consistent(name):
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from conftest import read_pool

    rows = read_pool(name)
    assert len(rows) in (1024, 256)
    for i, r in rows.items():
        assert sum(r["levels"]) == r["states"] and r["levels"][0] == 1, (name, i)
        assert r["deadlocks"] > 0 or r["dead_digest"] == (0, 0)
    # a few rows recomputed by the hash-set oracle
    nets = (W.batch_networks(1024, 11)[0] if name.startswith("batch")
            else W.served_networks(256, 5)[0])
    small = sorted((r["states"], i) for i, r in rows.items())[:5]
    for _, i in small:
        a = oracle.explore(nets[i])
        assert a.levels.tolist() == rows[i]["levels"] and a.n_transitions == rows[i]["transitions"]


def test_token_ring_golden_matches_table1(golden_dir):
    printed = dict(_read_table("token_ring_table1.txt"))
    for line in open(os.path.join(golden_dir, "token_ring_13_15.txt")):
        if line.startswith("#"):
            continue
        v = [int(x) for x in line.split()]
        assert v[1] == printed[v[0]] == sum(v[6:])
        assert v[3] == 0  # no deadlocks
