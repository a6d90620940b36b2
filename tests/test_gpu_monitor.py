"""GPU parity of gx_explore with a safety monitor (Sec. 3: the negation of a
safety property is an automaton added to the network) against the oracle's
monitored BFS: violating states, the first violating level, and with
stop_on_violation the levels, counts and table contents of the prefix the
exploration ends with, all bit-exact."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W
from paper_1801_05857_amd import models

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def _tick(n0, others, k):
    procs, mon = W.tick_counter(n0, others, k)
    files = {f"p{i}.aut": models.write_aut(*pr) for i, pr in enumerate(procs)}
    par = "par using in " + " || ".join(f'"p{i}.aut"' for i in range(len(procs))) + " end par"
    return models.add_monitor(models.parse_par(par, files), models.Lts(*mon), [k])


def _random(seed, P, ns, live, n_mon=4, bad=(3,)):
    net = W.random_lts(seed, P, ns, live, 3, 16, 0.25, 0.1)
    names = [f"R{r}" for r in range(net.rules.shape[0])] + \
        [f"L{l}" for l in range(net.rules.shape[0], net.n_labels)]
    mon = models.Lts(*W.random_monitor(seed, names, n_mon, 4))
    return models.add_monitor(net, mon, list(bad))


def _check(net, mp, bad, stop, B=32, G=4):
    want = oracle.explore(net, monitor=(mp, bad), stop_on_violation=stop)
    w = want.words
    full = oracle.explore(net, want_visited=False) if stop else want
    with gx.Table(w, B, max(64, 2 * full.n_states), subgroup=G, max_hashes=64) as t:
        for _ in range(2):  # the second run reuses the table's buffers
            t.clear()
            got = gx.explore(net, t, monitor=(mp, bad), stop_on_violation=stop)
            assert got.n_states == want.n_states
            assert got.levels.tolist() == want.levels.tolist()
            assert got.n_transitions == want.n_transitions
            assert np.array_equal(got.deadlocks, want.deadlocks)
            assert np.array_equal(got.violations, want.violations)
            assert got.violation_level == want.violation_level
        if stop and want.violation_level is not None:
            pre = oracle.explore(net, max_levels=want.violation_level + 1, want_visited=True)
            assert np.array_equal(t.dump(), pre.visited)
    return want


@pytest.mark.parametrize("stop", [False, True])
@pytest.mark.parametrize("n0,others,k", [(5, [3, 4], 7), (3, [5], 0), (6, [], 9),
                                         (8, [16, 16, 16, 4], 5)])
def test_tick_counter(dev, n0, others, k, stop):
    # the last case records 131072 violations: the record buffer grows and
    # the level is scanned again
    net, mp, bad = _tick(n0, others, k)
    want = _check(net, mp, bad, stop)
    assert want.violation_level == k


@pytest.mark.parametrize("stop", [False, True])
@pytest.mark.parametrize("seed,P,ns,live", [(1, 3, 8, 4), (2, 5, 8, 3), (3, 8, 16, 3),
                                            (4, 11, 64, 3), (5, 6, 32, 4)])
def test_random_networks(dev, seed, P, ns, live, stop):
    net, mp, bad = _random(seed, P, ns, live)
    _check(net, mp, bad, stop)


def test_monitor_that_never_fires(dev):
    net, mp, bad = _random(9, 5, 8, 4, bad=())
    want = _check(net, mp, bad, True)
    assert want.violations.shape[0] == 0 and want.violation_level is None


def test_bad_monitor_arguments(dev):
    net, mp, bad = _tick(4, [2], 2)
    with gx.Table(1, 32, 1024) as t:
        with pytest.raises(ValueError):
            gx.explore(net, t, monitor=(mp, bad[:-1]))
        with pytest.raises(ValueError):
            gx.explore(net, t, monitor=(len(net.n_states), bad))
