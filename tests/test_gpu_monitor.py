"""GPU parity of gx_explore with a safety monitor (Sec. 3: the negation of a
safety property is an automaton added to the network) against the oracle.

Both sides take the raw network and the automaton: the library composes them
(gx_network_add_monitor) and explores with the monitor scan; the oracle
watches the network with the automaton directly (oracle.explore_automaton).
Violating states, the first violating level, and with stop_on_violation the
levels, counts and table contents of the prefix the exploration ends with,
all bit-exact."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

from test_monitor_cpu import _tick_raw

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def _random(seed, P, ns, live, n_mon=4):
    net = W.random_lts(seed, P, ns, live, 3, 16, 0.25, 0.1)
    acts = list(range(net.rules.shape[0] + net.n_labels))
    return net, W.random_monitor(seed, acts, n_mon, 4)


def _check(net, aut, bad, stop, B=32, G=4):
    want = oracle.explore_automaton(net, aut, bad, stop_on_violation=stop)
    comp, mp, flags = gx.add_monitor(net, aut, bad)
    w = gx.network_words(comp)
    assert w == want.words
    full = oracle.explore_automaton(net, aut, bad) if stop else want
    with gx.Table(w, B, max(64, 2 * full.n_states), subgroup=G, max_hashes=64) as t:
        for _ in range(2):  # the second run reuses the table's buffers
            t.clear()
            got = gx.explore(comp, t, monitor=(mp, flags), stop_on_violation=stop)
            assert got.n_states == want.n_states
            assert got.levels.tolist() == want.levels.tolist()
            assert got.n_transitions == want.n_transitions
            assert np.array_equal(got.deadlocks, want.deadlocks)
            assert np.array_equal(got.violations, want.violations)
            assert got.violation_level == want.violation_level
        if stop and want.violation_level is not None:
            pre = oracle.explore_automaton(net, aut, bad, max_levels=want.violation_level + 1,
                                           want_visited=True)
            assert np.array_equal(t.dump(), pre.visited)
    return want


@pytest.mark.parametrize("stop", [False, True])
@pytest.mark.parametrize("n0,others,k", [(5, [3, 4], 7), (3, [5], 0), (6, [], 9),
                                         (8, [16, 16, 16, 4], 5)])
def test_tick_counter(dev, n0, others, k, stop):
    # the last case records 131072 violations: the record buffer grows and
    # the level is scanned again
    net, aut = _tick_raw(n0, others, k)
    want = _check(net, aut, [k], stop)
    assert want.violation_level == k


@pytest.mark.parametrize("stop", [False, True])
@pytest.mark.parametrize("seed,P,ns,live", [(1, 3, 8, 4), (2, 5, 8, 3), (3, 8, 16, 3),
                                            (4, 11, 64, 3), (5, 6, 32, 4)])
def test_random_networks(dev, seed, P, ns, live, stop):
    net, aut = _random(seed, P, ns, live)
    _check(net, aut, [3], stop)


def test_monitor_that_never_fires(dev):
    net, aut = _random(9, 5, 8, 4)
    want = _check(net, aut, [], True)
    assert want.violations.shape[0] == 0 and want.violation_level is None


def test_bad_monitor_arguments(dev):
    net, aut = _tick_raw(4, [2], 2)
    comp, mp, bad = gx.add_monitor(net, aut, [2])
    with gx.Table(1, 32, 1024) as t:
        with pytest.raises(ValueError):
            gx.explore(comp, t, monitor=(mp, bad[:-1]))
        with pytest.raises(ValueError):
            gx.explore(comp, t, monitor=(len(comp.n_states), bad))
