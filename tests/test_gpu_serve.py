"""GPU parity of the exploration server: every request served in a mix of
concurrent requests gives the oracle's result (and the result it gets alone),
bit-exact; admission waits when the HBM budget is held; too-small declared
bounds are retried; requests that can never fit are refused."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

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
    return nets, [oracle.explore(n) for n in nets]


def _same(got, ref):
    assert got.n_states == ref.n_states
    assert got.levels.tolist() == ref.levels.tolist()
    assert got.n_transitions == ref.n_transitions
    assert np.array_equal(got.deadlocks, ref.deadlocks)


def test_served_mix_equals_oracle(dev, reqs):
    nets, want = reqs
    with gx.Server(8 << 30, max_hashes=32) as srv:
        ids = [srv.submit(n, max(16, 2 * r.n_states)) for n, r in zip(nets, want)]
        for rid, ref in zip(ids, want):
            st, got, lat = srv.poll(rid)
            assert st == gx.GX_OK
            _same(got, ref)
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
