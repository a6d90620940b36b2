"""GPU parity of the exploration server: every request served in a mix of
concurrent requests gives the oracle's result (and the result it gets alone),
bit-exact; admission waits when the HBM budget is held; too-small declared
bounds are retried; requests that can never fit are refused."""
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


def _nets():
    nets = [W.fig1_producer_consumers(), W.tiny_cycles()]
    nets += [W.token_ring(n) for n in range(3, 12)]
    for seed in range(16):
        rng = W.SplitMix64(77 + seed)
        P = 3 + rng.below(8)
        nets.append(W.random_lts(77 + seed, P, 4 + rng.below(61), 2 + rng.below(3), 2, 32, 0.25,
                                 0.2 if seed % 2 else 0.0))
    # three- and four-word vectors, and networks with deadlocks
    nets += [W.random_lts(303, 12, 64, 3, 3, 32, 0.25, 0.1),
             W.random_lts(404, 16, 64, 2, 3, 32, 0.25, 0.0)]
    nets += [W.random_lts(s, 3 + s % 3, 8, 6, 2, 8, 0.5, 0.4) for s in (2, 8, 13, 14, 24)]
    nets.append(W.wide_rule(5, 4))  # one state with 1024 successors, all deadlocks
    nets += list(W.degenerate_networks().values())  # one-state processes, no transitions
    return nets


@pytest.fixture(scope="module")
def reqs():
    nets = _nets()
    return nets, [oracle.explore(n, want_visited=True) for n in nets]


def _same(got, ref):
    assert got.n_states == ref.n_states
    assert got.levels.tolist() == ref.levels.tolist()
    assert got.n_transitions == ref.n_transitions
    assert np.array_equal(got.deadlocks, ref.deadlocks)


def test_served_mix_equals_oracle(dev, reqs):
    nets, want = reqs
    with gx.Server(8 << 30, max_hashes=32, keep_states=True) as srv:
        ids = [srv.submit(n, max(16, 2 * r.n_states)) for n, r in zip(nets, want)]
        for rid, ref in zip(ids, want):
            st, got, lat = srv.poll(rid)
            assert st == gx.GX_OK
            _same(got, ref)
            # the request's table held exactly the reachable set
            assert np.array_equal(got.states, ref.visited)
            assert lat > 0
        s = srv.stats()
        assert s["completed"] == len(nets) and s["failed"] == 0
        assert s["active_peak"] > 1  # requests really overlapped on the device


@pytest.mark.parametrize("B,G,U", [(16, 4, 1), (32, 4, 2), (64, 16, 2)])
def test_served_mix_explicit_configurations(dev, reqs, B, G, U):
    nets, want = reqs
    with gx.Server(8 << 30, max_hashes=32, bucket_words=B, subgroup=G,
                   keys_per_subgroup=U) as srv:
        ids = [srv.submit(n, max(16, 2 * r.n_states)) for n, r in zip(nets, want)]
        for rid, ref in zip(ids, want):
            st, got, _ = srv.poll(rid)
            assert st == gx.GX_OK
            _same(got, ref)


def test_small_budget_queues_and_still_serves_all(dev, reqs):
    nets, want = reqs
    # room for only a few requests at a time (the largest reservation, the
    # 11-node ring, is about 268 MB): admission must wait for releases
    with gx.Server(400 << 20, max_hashes=32) as srv:
        ids = [srv.submit(n, max(16, 2 * r.n_states)) for n, r in zip(nets, want)]
        for rid, ref in zip(ids, want):
            st, got, _ = srv.poll(rid)
            assert st == gx.GX_OK
            _same(got, ref)
        assert srv.stats()["reserved_peak"] <= 400 << 20


def test_understated_bounds_are_retried(dev, reqs):
    nets, want = reqs
    with gx.Server(8 << 30, max_hashes=4) as srv:
        ids = [srv.submit(n, 8) for n in nets[:11]]  # far too small for most
        for rid, ref in zip(ids, want[:11]):
            st, got, _ = srv.poll(rid)
            assert st == gx.GX_OK
            _same(got, ref)
        assert srv.stats()["retried"] > 0


def test_request_larger_than_budget_is_refused(dev):
    with gx.Server(1 << 20) as srv:
        rid = srv.submit(W.token_ring(4), 10**9)
        st, got, _ = srv.poll(rid)
        assert st == gx.GX_ENOMEM and got is None


def test_poll_without_wait(dev):
    with gx.Server(1 << 30) as srv:
        rid = srv.submit(W.token_ring(9), 300000)
        r = srv.poll(rid, wait=False)
        while r is None:
            r = srv.poll(rid, wait=False)
        assert r[0] == gx.GX_OK and r[1].n_states == 118098


def test_served_pool_sample_matches_oracle(dev):
    """Requests of the served workload's pool (random networks, 1- to 4-word
    vectors, each declaring the product of its live-state counts), a seeded
    sample of 48 of those up to 2e7 states submitted at once, each result
    against the oracle's (tests/golden/served_pool.txt), then the same
    requests one at a time: each result is the same alone and in the mix."""
    nets, _, bounds = W.served_networks(256, 5)
    want = read_pool("served_pool.txt")
    small = [i for i in range(256) if want[i]["states"] <= 20_000_000]
    rng = W.SplitMix64(48)
    pick = [small[rng.below(len(small))] for _ in range(48)]
    assert {want[i]["words"] for i in pick} == {1, 2, 3, 4}

    def check(st, got, ref):
        assert st == gx.GX_OK
        assert got.n_states == ref["states"]
        assert got.levels.tolist() == ref["levels"]
        assert got.n_transitions == ref["transitions"]
        assert len(got.deadlocks) == ref["deadlocks"]
        assert oracle.digest(got.deadlocks, got.words_per_state) == ref["dead_digest"]

    with gx.Server(64 << 30, max_hashes=16) as srv:
        ids = [srv.submit(nets[i], bounds[i]) for i in pick]
        mix = []
        for rid, i in zip(ids, pick):
            st, got, _ = srv.poll(rid)
            check(st, got, want[i])
            mix.append(got)
        assert srv.stats()["active_peak"] > 1
        for i, m in zip(pick[:12], mix[:12]):
            st, got, _ = srv.poll(srv.submit(nets[i], bounds[i]))
            check(st, got, want[i])
            assert np.array_equal(got.deadlocks, m.deadlocks)
