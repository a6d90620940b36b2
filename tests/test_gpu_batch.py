"""GPU parity of batched exploration (many networks explored together: the
stepped schedule, and the persistent one with and without a hipGraph) against
the oracle BFS, instance by instance, bit-exact: counts, levels, deadlocks and
(keep_states) every instance's table contents; the benchmarked 1024-network
batch against the oracle's results of all its instances
(tests/golden/batch_1024_s11.txt)."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

from conftest import read_pool

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def _mixed_networks(k):
    nets = [W.fig1_producer_consumers(), W.tiny_cycles(), W.token_ring(5), W.token_ring(11),
            W.wide_rule(5, 4)]
    # networks with reachable deadlocks
    nets += [W.random_lts(s, 3 + s % 3, 8, 6, 2, 8, 0.5, 0.4) for s in (2, 8, 13, 14, 24)]
    for seed in range(k):
        rng = W.SplitMix64(1000 + seed)
        P = 3 + rng.below(8)
        ns = 4 + rng.below(61)
        live = 2 + rng.below(4)
        nets.append(W.random_lts(1000 + seed, P, ns, live, 2 + rng.below(2), 32, 0.25,
                                 0.15 if seed % 3 == 0 else 0.0))
    return nets


@pytest.fixture(scope="module")
def mixed():
    nets = _mixed_networks(28)
    want = [oracle.explore(n, want_visited=True) for n in nets]
    return nets, want


def _check(res, want, states=False):
    assert len(res) == len(want)
    for k, ((st, got), ref) in enumerate(zip(res, want)):
        assert st == gx.GX_OK, (k, gx.status_str(st))
        assert got.n_states == ref.n_states, k
        assert got.levels.tolist() == ref.levels.tolist(), k
        assert got.n_transitions == ref.n_transitions, k
        assert np.array_equal(got.deadlocks, ref.deadlocks), k
        if states:  # the instance's table holds exactly the reachable set
            assert np.array_equal(got.states, ref.visited), k


SCHEDULES = {"stepped": {}, "persistent": {"persistent": True}, "graph": {"use_graph": True}}


@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_batch_matches_oracle(dev, mixed, schedule):
    nets, want = mixed
    cap = [max(64, 3 * r.n_states) for r in want]
    with gx.Batch(nets, cap, max_hashes=32, keep_states=True, **SCHEDULES[schedule]) as b:
        b.run()
        _check(b.results(), want, states=True)
        # a second run resets every table and repeats the batch
        b.run()
        _check(b.results(), want, states=True)


@pytest.mark.parametrize("schedule", ["stepped", "graph"])
def test_benchmarked_batch_matches_oracle(dev, schedule):
    """The 1024-network batch exactly as the benchmark runs it (capacities
    twice the live-state products, autotuned configurations, 16 hash
    functions; the stepped schedule, and the persistent one from its
    hipGraph): every instance equals the oracle's exploration."""
    nets, bounds = W.batch_networks(1024, 11)
    want = read_pool("batch_1024_s11.txt")
    with gx.Batch(nets, [2 * c for c in bounds], max_hashes=16, **SCHEDULES[schedule]) as b:
        b.run()
        res = b.results()
    for i, (st, got) in enumerate(res):
        ref = want[i]
        assert st == gx.GX_OK, (i, gx.status_str(st))
        assert got.n_states == ref["states"], i
        assert got.levels.tolist() == ref["levels"], i
        assert got.n_transitions == ref["transitions"], i
        assert len(got.deadlocks) == ref["deadlocks"], i
        assert oracle.digest(got.deadlocks, got.words_per_state) == ref["dead_digest"], i


@pytest.mark.parametrize("schedule", ["stepped", "persistent"])
def test_batch_deeper_than_512_levels(dev, schedule):
    """A single 1500-state cycle: 1500 BFS levels (1500 steps, or one queue
    entry each)."""
    net = W.independent_cycles((1500,))
    want = oracle.explore(net, want_visited=True)
    assert len(want.levels) == 1500
    _check(gx.explore_batch([net], [4096], max_hashes=32, **SCHEDULES[schedule]), [want])
    # more levels than max_levels: the instance reports GX_ENOMEM
    res = gx.explore_batch([net], [4096], max_hashes=32, max_levels=1000, **SCHEDULES[schedule])
    assert res[0][0] == gx.GX_ENOMEM
    # exactly max_levels levels fit
    _check(gx.explore_batch([net], [4096], max_hashes=32, max_levels=1500,
                            **SCHEDULES[schedule]), [want])


def test_batch_degenerate_networks(dev):
    """One-state processes, no transitions, a rule that never fires, zero rules."""
    nets = list(W.degenerate_networks().values())
    nets += [W.independent_cycles((3, 5)), W.fig1_producer_consumers()]
    want = [oracle.explore(n) for n in nets]
    _check(gx.explore_batch(nets, [64] * len(nets), max_hashes=32), want)


@pytest.mark.parametrize("B,G,U", [(8, 8, 1), (16, 16, 2), (64, 8, 2), (32, 16, 1),
                                   (8, 4, 2), (16, 4, 1), (32, 4, 2)])
def test_batch_explicit_configurations(dev, mixed, B, G, U):
    nets, want = mixed
    cap = [max(64, 4 * r.n_states) for r in want]
    res = gx.explore_batch(nets, cap, bucket_words=B, subgroup=G, keys_per_subgroup=U,
                           max_hashes=64)
    _check(res, want)


def test_explicit_subgroup_of_four_caps_autotuned_bucket(dev, mixed):
    nets, want = mixed
    cap = [max(64, 4 * r.n_states) for r in want]
    with gx.Batch(nets, cap, subgroup=4, max_hashes=64) as b:
        for i in range(len(nets)):
            B, G, U = b.instance_config(i)
            assert G == 4 and B <= 32 and U == 1
        b.run()
        _check(b.results(), want)


def test_batch_equals_single_explorations(dev, mixed):
    nets, want = mixed
    cap = [max(64, 3 * r.n_states) for r in want]
    res = gx.explore_batch(nets, cap, max_hashes=32)
    for net, (st, got), c in zip(nets, res, cap):
        B, G, U = 32, 8, 1
        with gx.Table(gx.network_words(net), B, c, subgroup=G, keys_per_subgroup=U,
                      max_hashes=32) as t:
            alone = gx.explore(net, t)
        assert st == gx.GX_OK
        assert alone.n_states == got.n_states
        assert alone.levels.tolist() == got.levels.tolist()
        assert np.array_equal(alone.deadlocks, got.deadlocks)


@pytest.mark.parametrize("schedule", ["stepped", "persistent"])
def test_batch_isolates_a_failing_instance(dev, schedule):
    nets = [W.token_ring(6), W.token_ring(8), W.fig1_producer_consumers()]
    want = [oracle.explore(n) for n in nets]
    cap = [3 * want[0].n_states, 64, 64]  # the 34992-state ring gets 64 slots
    res = gx.explore_batch(nets, cap, max_hashes=4, **SCHEDULES[schedule])
    assert res[0][0] == gx.GX_OK and res[0][1].n_states == want[0].n_states
    assert res[1][0] == gx.GX_ETABLEFULL and res[1][1] is None
    assert res[2][0] == gx.GX_OK and res[2][1].n_states == 8


def test_batch_of_many_small_instances(dev):
    nets = [W.random_lts(5000 + s, 4, 8, 3, 2, 16, 0.3, 0.2) for s in range(300)]
    want = [oracle.explore(n) for n in nets]
    res = gx.explore_batch(nets, [max(64, 4 * r.n_states) for r in want], max_hashes=32)
    _check(res, want)


def test_autotune_returns_a_valid_configuration(dev):
    for w in (1, 2, 3):
        B, G, U = gx.autotune(w, 0.5)
        assert B in (8, 16, 32, 64) and G in (4, 8, 16) and U in (1, 2)
        assert G != 4 or B <= 32  # a 4-lane subgroup covers at most 32 words
        assert gx.autotune(w, 0.5) == (B, G, U)  # cached


def _size_class(cap):
    return 0 if cap <= 1 << 16 else 1 if cap <= 1 << 20 else 2 if cap <= 1 << 24 else 3


def test_autotune_per_size_class(dev):
    """Picks per (words, table size class), cached, with the timings behind
    them; the default B16-G4 is kept unless beaten by more than 3%."""
    for w in (1, 2):
        for cap in (1 << 12, 1 << 18, 1 << 22):
            t = gx.autotune_capacity(w, cap)
            assert t["size_class"] == _size_class(cap)
            assert t["keys_per_subgroup"] == 1 and t["candidates"] >= 8
            assert t["bucket_words"] in (8, 16, 32, 64) and t["subgroup"] in (4, 8, 16)
            assert t["ns_per_key"] > 0 and t["ns_per_key_default"] > 0
            assert t["ns_per_key_runner_up"] > 0
            if (t["bucket_words"], t["subgroup"]) != (16, 4):
                assert t["ns_per_key"] * 1.03 < t["ns_per_key_default"]
            else:
                assert t["ns_per_key"] == t["ns_per_key_default"]
            assert gx.autotune_capacity(w, cap) == t  # cached
            # any capacity of the same class gets the same pick
            assert gx.autotune_capacity(w, cap - 1) == t


def test_batch_tunes_for_the_combined_footprint(dev):
    """An instance's autotuned configuration is the pick for its words and the
    combined capacity of the batch's instances of its slot width."""
    # 810, 34992, 1299078 and 8 reachable states (one-, one-, two- and
    # one-word vectors)
    nets = [W.token_ring(5), W.token_ring(8), W.token_ring(11), W.fig1_producer_consumers()]
    caps = [1 << 11, 1 << 17, 1 << 22, (1 << 24) + 1]
    words = [gx.network_words(nt) for nt in nets]
    assert words == [1, 1, 2, 1]
    total = {}
    for w, c in zip(words, caps):
        total[w] = total.get(w, 0) + c
    with gx.Batch(nets, caps, max_hashes=32) as b:
        for i, w in enumerate(words):
            t = gx.autotune_capacity(w, total[w])
            assert b.instance_config(i) == (t["bucket_words"], t["subgroup"], 1)
        b.run()
        _check(b.results(), [oracle.explore(n) for n in nets])
