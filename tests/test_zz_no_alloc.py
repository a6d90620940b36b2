"""gx_explore_noalloc (exploration with the library's static scratch array,
for callers that cannot allocate) against gx_explore on the same networks:
two calls in a row, the second with a smaller network, each bit-exact in
level counts, transitions, deadlocks and table contents; and the size
limits reported as GX_ENOMEM."""
import numpy as np
import pytest

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


def _reference(net, B, cap):
    with gx.Table(gx.network_words(net), B, cap, max_hashes=32) as t:
        r = gx.explore(net, t)
        return r, t.dump()


def _check(net, B, cap):
    want, want_dump = _reference(net, B, cap)
    with gx.Table(gx.network_words(net), B, cap, max_hashes=32) as t:
        got = gx.explore_noalloc(net, t)
        assert got.n_states == want.n_states
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want_dump)
    return got


def test_two_calls_in_a_row_second_smaller(dev):
    # first: three-word states (four-word slots), 248,832 states, levels up
    # to about 30,000 states
    big = W.large_random_network(live=4)
    r1 = _check(big, 16, 2 * 248832)
    assert r1.n_states == 248832
    # second: a smaller one-word network with deadlocks, in the scratch the
    # first call left behind
    small = W.random_lts(8, 4, 8, 6, 2, 8, 0.5, 0.4)
    r2 = _check(small, 32, 4096)
    assert r2.n_states < r1.n_states and len(r2.deadlocks) > 0


def test_repeated_calls_and_word_widths(dev):
    for net, B, cap in ((W.tiny_cycles(), 32, 1 << 16), (W.token_ring(11), 16, 4 * 1299078),
                        (W.fig1_producer_consumers(), 8, 64), (W.tiny_cycles(), 4, 1 << 14)):
        _check(net, B, cap)


def test_limits_are_enomem(dev):
    net = W.tiny_cycles()  # 21 levels
    with gx.Table(1, 32, 1 << 16) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore_noalloc(net, t, max_levels=5)
        assert e.value.code == gx.GX_ENOMEM
    dl = W.wide_rule(4, 4)  # 256 deadlocks
    with gx.Table(gx.network_words(dl), 16, 1024) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore_noalloc(dl, t, max_deadlocks=100)
        assert e.value.code == gx.GX_ENOMEM
    # a level beyond the scratch frontier (2,095,072 two-word states): the
    # 15-node token ring reaches levels of about 2.1 million states
    ring = W.token_ring(15)
    with gx.Table(2, 16, 2 * 143489070, max_hashes=32) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore_noalloc(ring, t)
        assert e.value.code == gx.GX_ENOMEM


def test_monitor_rejected(dev):
    net = W.tiny_cycles()
    with gx.Table(1, 32, 1 << 16) as t:
        opts = gx._ExploreOpts(0, 0, None, 0, 0, 0, 0, np.ones(8, np.uint8).ctypes.data)
        h = gx._NetHolder(net)
        levels = np.zeros(64, np.uint64)
        summ = gx._ExploreSummary()
        import ctypes
        code = gx.lib().gx_explore_noalloc(ctypes.byref(h.c), t.handle, ctypes.byref(opts),
                                           levels.ctypes.data, 64, None, 0, ctypes.byref(summ))
        assert code == gx.GX_EINVAL
