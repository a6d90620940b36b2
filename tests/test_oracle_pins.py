"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

Every test here checks the oracle against something other than itself: the
worked example and printed counts of the paper, closed forms of networks whose
reachable product is known analytically, hand-packed vectors, an independent
library routine (numpy) and a brute-force fixpoint enumerator.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads as W

from conftest import GOLDEN


def _read_kv(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            out[k] = int(v)
    return out


def _read_table(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append(tuple(int(x) for x in line.split()))
    return rows


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ------------------------------------------------------------ Fig. 1 (Sec. 3)
def test_fig1_state_and_transition_counts():
    want = _read_kv("fig1_counts.txt")
    r = oracle.explore(W.fig1_producer_consumers(), want_visited=True)
    assert r.n_states == want["states"]
    assert r.n_transitions == want["transitions"]
    # every one of the 2*2*2 vectors is reachable
    assert r.visited.shape == (8, 1)


def test_fig1_sync_semantics_reading():
    # If send/rec could also fire alone, the count of 24 transitions would be
    # exceeded; dropping the rules leaves the rendezvous-only labels free.
    net = W.fig1_producer_consumers()
    free = W.Network(net.n_states, net.initial, net.trans, net.n_labels,
                     np.zeros((0, 3), np.int32))
    r = oracle.explore(free)
    assert r.n_transitions > 24


# ------------------------------------------------- Token Ring (Table 1, right)
def test_token_ring_closed_form_matches_table1():
    # the closed form 2N * 3^(N-1) reproduces every printed row of Table 1
    for n, states in _read_table("token_ring_table1.txt"):
        assert 2 * n * 3 ** (n - 1) == states


@pytest.mark.parametrize("n", range(2, 10))
def test_token_ring_counts(n):
    printed = dict(_read_table("token_ring_table1.txt"))
    r = oracle.explore(W.token_ring(n))
    assert r.n_states == printed[n]
    assert r.deadlocks.shape[0] == 0
    # 3 bits per node: one word up to 10 nodes (Sec. 5.2)
    assert r.words == 1


def test_token_ring_11_needs_two_words():
    w, *_ = oracle.pack_plan(W.token_ring(11).n_states)
    assert w == 2
    w, *_ = oracle.pack_plan(W.token_ring(10).n_states)
    assert w == 1


# ---------------------------------------------------------- closed forms
def _cycle_levels(sizes):
    poly = np.array([1], dtype=np.int64)
    for n in sizes:
        poly = np.convolve(poly, np.ones(n, dtype=np.int64))
    return poly


@pytest.mark.parametrize("sizes", [(8, 8, 8, 8), (3, 5, 7), (2,), (4, 1, 6), (16, 9)])
def test_independent_cycles(sizes):
    r = oracle.explore(W.independent_cycles(sizes))
    assert r.n_states == int(np.prod(sizes))
    assert r.levels.tolist() == _cycle_levels(sizes).tolist()
    # one tau step per process in every state
    assert r.n_transitions == int(np.prod(sizes)) * len(sizes)
    assert r.deadlocks.shape[0] == 0


def test_tiny_cycles_closed_form():
    # Each synchronised pair (a, b) moves a -> a+1, b -> b+1 (mod 8) freely and
    # jumps (0, 0) -> (4, 4) jointly; its distance from (0, 0) is a + b, or
    # a + b - 7 when both a, b >= 4.  The two pairs are independent, so the
    # level counts are the self-convolution of one pair's distance histogram.
    dist = np.zeros(15, dtype=np.int64)
    for a in range(8):
        for b in range(8):
            d = a + b
            if a >= 4 and b >= 4:
                d = min(d, a + b - 7)
            dist[d] += 1
    dist = np.trim_zeros(dist, "b")
    levels = np.convolve(dist, dist)
    r = oracle.explore(W.tiny_cycles())
    assert r.n_states == 4096
    assert r.levels.tolist() == levels.tolist()
    # 4 tau steps everywhere, plus one joint jump where a pair sits at (0, 0)
    assert r.n_transitions == 4 * 4096 + 64 + 64
    assert r.deadlocks.shape[0] == 0


# ---------------------------------------------------------- packing
def _packing_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "packing_examples.txt")):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        ns, loc, words = (part.strip() for part in line.split("|"))
        rows.append(([int(x) for x in ns.split(",")], [int(x) for x in loc.split(",")],
                     [int(x, 16) for x in words.split(",")]))
    return rows


@pytest.mark.parametrize("ns,loc,words", _packing_rows())
def test_packing_examples(ns, loc, words):
    got = oracle.pack(ns, [loc])[0]
    assert got.tolist() == words
    assert all(x >> 31 == 0 for x in got.tolist())


def test_packing_rejects_oversized_field():
    with pytest.raises(ValueError):
        oracle.pack_plan([2**31 + 1])
    with pytest.raises(ValueError):
        oracle.pack_plan([0, 4])


# ---------------------------------------------------------- brute force
def _tiny_random(seed):
    rng = W.SplitMix64(seed)
    P = 2 + rng.below(3)
    ns = [2 + rng.below(6) for _ in range(P)]
    live = [max(1, n - rng.below(2)) for n in ns]
    return W.random_lts(seed, P, ns, live, out_degree=1 + rng.below(3), n_labels=6,
                        rendezvous_frac=0.34, sink_prob=0.25)


@pytest.mark.parametrize("seed", range(30))
def test_bfs_equals_bruteforce(seed):
    net = _tiny_random(seed)
    a = oracle.explore(net, want_visited=True)
    b = oracle.bruteforce(net, want_visited=True)
    assert a.n_states == b.n_states
    assert a.n_transitions == b.n_transitions
    assert a.levels.tolist() == b.levels.tolist()
    assert np.array_equal(a.deadlocks, b.deadlocks)
    assert np.array_equal(a.visited, b.visited)


def test_bruteforce_on_fig1_and_tiny():
    b = oracle.bruteforce(W.fig1_producer_consumers())
    assert (b.n_states, b.n_transitions) == (8, 24)
    b = oracle.bruteforce(W.tiny_cycles())
    assert b.n_states == 4096 and b.n_transitions == 16512


def test_deadlocks_are_states_without_successors():
    # a chain 0 -> 1 -> 2 in one process, 2 is terminal; a 2-cycle in another
    net = W.Network(np.array([3, 2], np.uint32), np.array([0, 0], np.uint32),
                    [np.array([[0, 0, 1], [1, 0, 2]], np.uint32),
                     np.array([[0, 1, 1], [1, 1, 0]], np.uint32)],
                    2, np.array([[-1, 1]], np.int32))
    r = oracle.explore(net, want_visited=True)
    # process 1 only moves through the one-participant rule, so never blocks
    assert r.n_states == 6 and r.deadlocks.shape[0] == 0
    net.rules = np.array([[0, 1]], np.int32)  # now both must step together
    r = oracle.explore(net, want_visited=True)
    # label 0 of p0 and label 1 of p1 are governed: (0,0)->(1,1)->(2,0), stuck
    assert r.n_states == 3
    assert r.levels.tolist() == [1, 1, 1]
    assert r.deadlocks.tolist() == [[2 | (0 << 2)]]


@pytest.mark.parametrize("seed", range(5))
def test_levels_partition_the_visited_set(seed):
    net = _tiny_random(seed)
    r = oracle.explore(net, want_visited=True)
    assert int(r.levels.sum()) == r.n_states == r.visited.shape[0]
    assert r.levels[0] == 1 and (r.levels > 0).all()
    # the dump holds no duplicates and is sorted
    assert np.unique(r.visited, axis=0).shape[0] == r.n_states


# ---------------------------------------------------------- find-or-put oracle
@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_set_insert_matches_numpy_unique(w):
    rng = np.random.default_rng(w)
    base = rng.integers(0, 2**31 - 1, size=(500, w), dtype=np.uint32)
    keys = base[rng.integers(0, 500, size=4000)]
    s = oracle.OracleSet(w)
    status, n_new = s.insert(keys)
    uniq, first = np.unique(keys, axis=0, return_index=True)
    want = np.zeros(keys.shape[0], np.uint8)
    want[first] = 1
    assert n_new == uniq.shape[0] == len(s)
    assert np.array_equal(status, want)
    assert np.array_equal(s.dump(), uniq)  # np.unique sorts lexicographically
    # a second pass finds everything
    status2, n_new2 = s.insert(keys)
    assert n_new2 == 0 and not status2.any()
    assert s.contains(keys[0]) and len(s) == uniq.shape[0]


def test_duplicated_stream_shape():
    ks = W.duplicated_stream(1000, 3, 2, seed=5)
    uniq, counts = np.unique(ks, axis=0, return_counts=True)
    assert uniq.shape[0] == 1000 and (counts == 3).all()
    assert not (ks == 0xFFFFFFFF).any()


def test_fig1_successors_by_hand():
    """oracle.successors against successor multisets derived by hand from
    Fig. 1 (tests/golden/fig1_successors.txt)."""
    net = W.fig1_producer_consumers()
    rows = []
    for line in open(os.path.join(GOLDEN, "fig1_successors.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        state, succ = line.split(":")
        rows.append((int(state, 16), sorted(int(x, 16) for x in succ.split())))
    counts, succ = oracle.successors(net, np.array([[s] for s, _ in rows], dtype=np.uint32))
    assert counts.tolist() == [len(want) for _, want in rows]
    at = 0
    for (_, want), c in zip(rows, counts):
        assert sorted(succ[at:at + int(c), 0].tolist()) == want
        at += int(c)


def test_successor_counts_sum_to_transitions():
    """Over the reachable set, successor counts add up to the transition count
    of the BFS, and the successors of the deadlocks are empty (random networks
    with deadlocks, and the Token Ring)."""
    for net in [W.random_lts(s, 3 + s % 3, 8, 6, 2, 8, 0.5, 0.4) for s in (2, 8, 13)] + \
            [W.token_ring(5)]:
        r = oracle.explore(net, want_visited=True)
        counts, succ = oracle.successors(net, r.visited)
        assert int(counts.sum()) == r.n_transitions
        assert succ.shape[0] == r.n_transitions
        if len(r.deadlocks):
            dc, _ = oracle.successors(net, r.deadlocks)
            assert (dc == 0).all()
        # closure: every successor is in the reachable set
        vis = {tuple(v) for v in r.visited.tolist()}
        assert all(tuple(v) in vis for v in succ.tolist())


def test_bfs_prefix_matches_full_search():
    """explore(max_levels=k) gives the first k level counts of the full BFS
    and stops before expanding level k-1 (fewer transitions counted), unless
    the search ends first."""
    for net in [W.token_ring(7), W.tiny_cycles(), W.large_random_network(live=3)]:
        full = oracle.explore(net)
        for k in (1, 2, 5, len(full.levels), len(full.levels) + 3):
            pre = oracle.explore(net, max_levels=k)
            assert pre.levels.tolist() == full.levels[:k].tolist()
            if k <= len(full.levels):  # the last known level is not expanded
                assert pre.n_transitions < full.n_transitions
            else:
                assert pre.n_transitions == full.n_transitions


@pytest.mark.parametrize("P,k", [(2, 3), (4, 4), (6, 5)])
def test_wide_rule_closed_form(P, k):
    """One rule over every process, k choices each: the initial state has k^P
    successors, all deadlocks (closed form)."""
    r = oracle.explore(W.wide_rule(P, k))
    assert r.n_states == 1 + k ** P
    assert r.n_transitions == k ** P
    assert r.levels.tolist() == [1, k ** P]
    assert len(r.deadlocks) == k ** P


# (n_states, levels, transitions, deadlocks), each derived by hand from the
# synchronous product's definition (Sec. 3)
DEGENERATE = {
    "lone": (1, [1], 0, 1),      # no transition at all: the initial state is stuck
    "selfloop": (1, [1], 1, 0),  # the loop is a transition back to the same state
    "ones": (1, [1], 0, 1),
    "never": (1, [1], 0, 1),     # a label named in a rule never fires alone
    "chain": (3, [1, 1, 1], 5, 0),  # 3 self-loops + 2 chain steps; loops prevent deadlock
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_degenerate_networks(name):
    net = W.degenerate_networks()[name]
    n, levels, trans, dead = DEGENERATE[name]
    r = oracle.explore(net)
    assert r.n_states == n
    assert r.levels.tolist() == levels
    assert r.n_transitions == trans
    assert len(r.deadlocks) == dead
    if dead:
        assert r.deadlocks.tolist() == [[0] * r.words]  # the all-initial vector packs to 0
