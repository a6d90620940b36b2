"""GPU parity of gx_explore against the oracle BFS: reachable-state count,
per-level counts, transition count, deadlock set and the final table contents,
all bit-exact."""
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


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def _read_rows(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append(tuple(int(x) for x in line.split()))
    return rows


def _explore_and_compare(net, B=32, G=0, cap=None, check_dump=True, **kw):
    want = oracle.explore(net, want_visited=check_dump)
    w = want.words
    cap = cap or max(64, 2 * want.n_states)
    # buckets of 2 or 4 slots at load 0.5 can exhaust 8 hash functions
    kw.setdefault("max_hashes", 64)
    with gx.Table(w, B, cap, subgroup=G, **kw) as t:
        got = gx.explore(net, t)
        assert got.words_per_state == w
        assert got.n_states == want.n_states
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        if check_dump:
            assert np.array_equal(t.dump(), want.visited)
        s = t.stats()
        assert s.stored == want.n_states and s.full == 0
    return got


def test_fig1(dev):
    got = _explore_and_compare(W.fig1_producer_consumers())
    assert (got.n_states, got.n_transitions) == (8, 24)


def test_tiny_cycles_config(dev):
    # the tiny configuration: one-word states, table of 2^16 words, buckets of 32
    got = _explore_and_compare(W.tiny_cycles(), B=32, cap=(1 << 16))
    assert got.n_states == 4096 and len(got.levels) == 21


@pytest.mark.parametrize("n", list(range(2, 13)))
def test_token_ring(dev, n):
    got = _explore_and_compare(W.token_ring(n), B=32)
    assert got.n_states == 2 * n * 3 ** (n - 1)


def _ring_golden():
    rows = {}
    for line in open(os.path.join(GOLDEN, "token_ring_13_15.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x) for x in line.split()]
        rows[v[0]] = {"states": v[1], "transitions": v[2], "deadlocks": v[3],
                      "digest": (v[4], v[5]), "levels": v[6:]}
    return rows


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_token_ring_large(dev, n):
    """Table 1 (right) beyond the hash-set oracle's reach: the state count
    printed in the paper (13..16 nodes, two-word vectors); for 13..15 nodes
    also every level count, the transition count and the digest of the
    table's contents from the oracle's dense BFS."""
    printed = dict(_read_rows("token_ring_table1.txt"))
    net = W.token_ring(n)
    with gx.Table(2, 16, 2 * printed[n], subgroup=4, keys_per_subgroup=1, max_hashes=32) as t:
        got = gx.explore(net, t)
        assert got.n_states == printed[n] == 2 * n * 3 ** (n - 1)
        assert len(got.deadlocks) == 0
        assert int(got.levels.sum()) == got.n_states
        assert t.stats().stored == got.n_states
        if n <= 15:
            ref = _ring_golden()[n]
            assert got.levels.tolist() == ref["levels"]
            assert got.n_transitions == ref["transitions"]
            assert table_digest(t, dev) == (ref["states"], ref["digest"])


@pytest.mark.parametrize("name", ["lone", "selfloop", "ones", "never", "chain"])
@pytest.mark.parametrize("B,G", [(4, 4), (32, 8)])
def test_degenerate_networks(dev, name, B, G):
    _explore_and_compare(W.degenerate_networks()[name], B=B, G=G)


@pytest.mark.parametrize("sizes", [(8, 8, 8, 8), (3, 5, 7, 11, 13), (2,) * 20, (64, 64, 64)])
def test_independent_cycles(dev, sizes):
    _explore_and_compare(W.independent_cycles(sizes), B=16)


SPECS = [(B, G) for B in (4, 8, 16, 32, 64) for G in (8, 16, 32, 64)]
SPECS += [(B, 4) for B in (4, 8, 16, 32)]  # 4-lane subgroups


def _net_for_words(w):
    # 1 word: 6 processes of 16 states; 2: 8 x 32; 3: 12 x 64; 4: 16 x 64
    if w == 1:
        return W.random_lts(101, 6, 16, 6, 3, 32, 0.25, 0.1)
    if w == 2:
        return W.random_lts(202, 8, 32, 4, 3, 32, 0.25, 0.1)
    if w == 3:
        return W.random_lts(303, 12, 64, 3, 3, 32, 0.25, 0.1)
    return W.random_lts(404, 16, 64, 2, 3, 32, 0.25, 0.0)


@pytest.mark.parametrize("w", [1, 2, 3, 4])
@pytest.mark.parametrize("B,G", SPECS, ids=[f"B{B}-G{G}" for B, G in SPECS])
def test_random_networks_every_specialisation(dev, w, B, G):
    net = _net_for_words(w)
    got = _explore_and_compare(net, B=B, G=G)
    assert got.words_per_state == w


@pytest.mark.parametrize("live,slice_states", [(2, 1), (3, 64)])
def test_tiny_slices(dev, live, slice_states):
    """Slices of one state (4,096-state network, levels up to 924 states,
    past the one-workgroup limit of a few hundred) and of 64 states (157,464
    states): a launch pair per slice."""
    net = W.random_lts(303, 12, 64, live, 3, 32, 0.25, 0.1)
    want = oracle.explore(net, want_visited=True)
    with gx.Table(want.words, 16, 2 * want.n_states, subgroup=4, max_hashes=64) as t:
        got = gx.explore(net, t, slice_states=slice_states)
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)


@pytest.mark.parametrize("slice_states", [0, 1000])
@pytest.mark.parametrize("B,G", [(16, 4), (32, 8)])
def test_four_word_states_through_both_kernels(dev, B, G, slice_states):
    """Four-word states with levels of up to 21,087 states, past the
    one-workgroup limit, so they take the generation and probe kernels: the
    successor buffer holds whole four-word slots there (three-word states
    hold three words; the w = 3 networks above cover those)."""
    net = W.random_lts(405, 16, 64, [3] * 4 + [2] * 12, 3, 32, 0.25, 0.0)
    want = oracle.explore(net, want_visited=True)
    assert want.words == 4 and max(want.levels) > 4096
    with gx.Table(4, B, 2 * want.n_states, subgroup=G, max_hashes=64) as t:
        got = gx.explore(net, t, slice_states=slice_states)
        assert got.n_states == want.n_states
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(t.dump(), want.visited)


@pytest.mark.parametrize("seed", [2, 8, 11, 13, 14, 20, 24, 25])
def test_random_networks_with_deadlocks(dev, seed):
    net = W.random_lts(seed, 3 + seed % 3, 8, 6, 2, 8, 0.5, 0.4)
    got = _explore_and_compare(net, B=16, G=16)
    assert got.deadlocks.shape[0] > 0


def test_larger_random_network(dev):
    # about 10^6 states; chunked staging (tiles with many successors)
    net = W.random_lts(7, 9, 64, 5, 4, 32, 0.25, 0.05)
    got = _explore_and_compare(net, B=32, G=32, check_dump=False)
    assert got.n_states > 100_000


def test_table_full_is_reported(dev):
    net = W.token_ring(8)  # 34992 states
    with gx.Table(1, 8, 4096, max_hashes=2) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore(net, t)
        assert e.value.code == gx.GX_ETABLEFULL
        # invariants still hold: what is stored is reachable and unique
        dump = t.dump()
        want = oracle.explore(net, want_visited=True).visited
        assert np.unique(dump, axis=0).shape[0] == dump.shape[0]
        assert np.isin(dump.view(np.uint32).ravel(), want.ravel()).all()


def test_frontier_overflow_is_reported(dev):
    net = W.token_ring(9)
    with gx.Table(1, 32, 1 << 18) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore(net, t, frontier_capacity=64)
        assert e.value.code == gx.GX_ENOMEM


def test_non_empty_table_rejected(dev):
    net = W.token_ring(4)
    with gx.Table(1, 32, 1024) as t:
        gx.explore(net, t)
        with pytest.raises(gx.GxError) as e:
            gx.explore(net, t)
        assert e.value.code == gx.GX_EINVAL
        t.clear()
        got = gx.explore(net, t)
        assert got.n_states == 216


def test_table_with_inserted_keys_rejected(dev):
    """A table that received keys through find-or-put is not empty: refused
    before any device work, accepted again once cleared."""
    net = W.token_ring(4)
    with gx.Table(1, 32, 1024) as t:
        keys = torch.tensor([[5]], dtype=torch.int32, device=dev)
        status = torch.empty(1, dtype=torch.uint8, device=dev)
        t.find_or_put(keys, status)
        with pytest.raises(gx.GxError) as e:
            gx.explore(net, t)
        assert e.value.code == gx.GX_EINVAL
        assert t.dump().shape[0] == 1  # untouched
        t.clear()
        assert gx.explore(net, t).n_states == 216


def test_word_count_mismatch_rejected(dev):
    with gx.Table(2, 32, 1024) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore(W.token_ring(4), t)
        assert e.value.code == gx.GX_EINVAL


def test_fig1_from_paper_syntax(dev, golden_dir):
    import os

    from paper_1801_05857_amd import models

    d = os.path.join(golden_dir, "fig1")
    files = {n: open(os.path.join(d, n)).read() for n in ("producer.aut", "consumer.aut")}
    net = models.parse_par(open(os.path.join(d, "network.exp")).read(), files)
    got = _explore_and_compare(net)
    assert (got.n_states, got.n_transitions) == (8, 24)


@pytest.mark.parametrize("which", ["tiny", "ring9", "w1", "w2", "w3", "w4"])
@pytest.mark.parametrize("B,G,U", [(32, 8, 1), (8, 16, 2)])
def test_local_duplicate_filter_keeps_results(dev, which, B, G, U):
    net = {"tiny": W.tiny_cycles(), "ring9": W.token_ring(9)}.get(which)
    if net is None:
        net = _net_for_words(int(which[1]))
    want = oracle.explore(net, want_visited=True)
    with gx.Table(want.words, B, max(64, 2 * want.n_states), subgroup=G, keys_per_subgroup=U,
                  max_hashes=64) as t:
        got = gx.explore(net, t, local_dedup=True)
        assert got.n_states == want.n_states
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)
        s = t.stats()
        # every successor is either probed or dropped as a local duplicate
        assert s.lookups + got.local_duplicates == want.n_transitions + 1
    if which in ("tiny", "ring9"):
        assert got.local_duplicates > 0


@pytest.mark.parametrize("P,k", [(4, 4), (6, 5)])
@pytest.mark.parametrize("dedup", [False, True])
def test_wide_rule_fan_out(dev, P, k, dedup):
    """One state with k^P successors (a rule over every process): slices of
    very different sizes, the general rule enumeration, many deadlocks."""
    net = W.wide_rule(P, k)
    want = oracle.explore(net, want_visited=True)
    with gx.Table(want.words, 32, 2 * want.n_states, subgroup=8, max_hashes=64) as t:
        got = gx.explore(net, t, local_dedup=dedup)
        assert got.n_states == want.n_states == 1 + k ** P
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)


@pytest.mark.parametrize("n", [1500, 130])
def test_long_chain_of_small_levels(dev, n):
    """n levels of one state each: small levels run on one workgroup, up to
    64 of them per launch, so the chain takes several launches."""
    got = _explore_and_compare(W.independent_cycles((n,)), B=16, cap=4 * n)
    assert len(got.levels) == n


def test_small_and_large_levels_alternate(dev):
    """Levels grow past the one-workgroup limit and shrink below it again
    (the large workload's family at 4 live states: 248,832 states, levels up
    to about 30,000), in every bucket size."""
    net = W.large_random_network(live=4)
    for B in (4, 16, 64):
        _explore_and_compare(net, B=B, check_dump=(B == 16))


@pytest.mark.parametrize("dedup", [False, True])
@pytest.mark.parametrize("slice_states,frontier", [(256, 0), (1000, 0), (700, 1 << 16)])
def test_many_slices_per_level(dev, dedup, slice_states, frontier):
    """Slices of a few hundred states cut the levels of the 248,832-state
    network (up to about 30,000 states) into many, their successor counters
    alternating; with a frontier capacity of 2^16 the room also runs out
    within levels and read-backs come between slices.  Three explorations in
    a row into one table."""
    net = W.large_random_network(live=4)
    want = oracle.explore(net, want_visited=True)
    with gx.Table(want.words, 16, 2 * want.n_states, max_hashes=64) as t:
        for _ in range(3):
            t.clear()
            got = gx.explore(net, t, frontier_capacity=frontier, local_dedup=dedup,
                             slice_states=slice_states)
            assert got.n_states == want.n_states
            assert got.levels.tolist() == want.levels.tolist()
            assert got.n_transitions == want.n_transitions
            assert np.array_equal(got.deadlocks, want.deadlocks)
            assert np.array_equal(t.dump(), want.visited)


@pytest.mark.parametrize("cap,ok", [(1, False), (255, False), (256, True)])
def test_deadlock_capacity(dev, cap, ok):
    """wide_rule(4, 4): 256 deadlocks, all in level 1."""
    net = W.wide_rule(4, 4)
    with gx.Table(gx.network_words(net), 16, 1024, max_hashes=32) as t:
        if ok:
            got = gx.explore(net, t, deadlock_capacity=cap)
            assert len(got.deadlocks) == 256
        else:
            with pytest.raises(gx.GxError) as e:
                gx.explore(net, t, deadlock_capacity=cap)
            assert e.value.code == gx.GX_ENOMEM


def test_explore_through_a_network_view(dev):
    """A network view built once serves repeated explorations."""
    net = W.token_ring(7)
    want = oracle.explore(net, want_visited=True)
    view = gx.network_view(net)
    with gx.Table(1, 32, 4 * want.n_states) as t:
        for _ in range(3):
            t.clear()
            got = gx.explore(view, t)
            assert got.levels.tolist() == want.levels.tolist()
            assert got.n_transitions == want.n_transitions
        assert np.array_equal(t.dump(), want.visited)
