"""Safety monitors (Sec. 3: the negation of a safety property is an automaton
added to the network; reaching one of its bad states is a violation).  The
oracle's monitored search is pinned to closed forms and to the brute-force
fixpoint enumerator; the composition helper to the unmonitored search."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_1801_05857_amd import models


def _compose(procs, mon, bad):
    files = {f"p{i}.aut": models.write_aut(*pr) for i, pr in enumerate(procs)}
    par = "par using in " + " || ".join(f'"p{i}.aut"' for i in range(len(procs))) + " end par"
    net = models.parse_par(par, files)
    return models.add_monitor(net, models.Lts(*mon), bad)


@pytest.mark.parametrize("n0,others,k", [(5, [3, 4], 7), (4, [2], 2), (3, [5], 0),
                                         (6, [], 9), (2, [2, 2, 3], 1)])
def test_tick_counter_closed_form(n0, others, k):
    # (process 0, automaton) reach the chain (m ticks, m mod n0) for m < k and
    # then every (k, p0): k + n0 states at distances 0, 1, ..., k + n0 - 1;
    # the other cycles are independent, so levels are the convolution of the
    # distance histograms, and the violations are the n0 * prod(others)
    # states with the automaton at k, first reached at distance k
    procs, mon = W.tick_counter(n0, others, k)
    net, mp, bad = _compose(procs, mon, [k])
    hist = np.ones(k + n0, dtype=np.int64)
    for n in others:
        hist = np.convolve(hist, np.ones(n, dtype=np.int64))
    prod = int(np.prod(others)) if others else 1
    r = oracle.explore(net, monitor=(mp, bad))
    assert r.levels.tolist() == hist.tolist()
    assert r.n_states == (k + n0) * prod
    assert r.violations.shape[0] == n0 * prod
    assert r.violation_level == k
    # stopping at the first violation: levels 0..k, one violating state
    s = oracle.explore(net, monitor=(mp, bad), stop_on_violation=True)
    assert s.levels.tolist() == hist[:k + 1].tolist()
    assert s.n_states == int(hist[:k + 1].sum())
    assert s.violations.shape[0] == 1 and s.violation_level == k


def test_unobserving_monitor_changes_nothing():
    # a one-state automaton that observes actions but never moves: the
    # composed network has the same states, levels and transitions
    net = W.random_lts(17, 4, 8, 4, 3, 16, 0.25, 0.2)
    names = [f"R{r}" for r in range(net.rules.shape[0])] + [f"L{l}" for l in range(net.n_labels)]
    mon = models.Lts(1, 0, [(0, a, 0) for a in names[::3]])
    comp, mp, bad = models.add_monitor(net, mon, [])
    a, b = oracle.explore(net), oracle.explore(comp, monitor=(mp, bad))
    assert a.levels.tolist() == b.levels.tolist()
    assert a.n_transitions == b.n_transitions
    assert b.violations.shape[0] == 0 and b.violation_level is None


@pytest.mark.parametrize("seed", range(6))
def test_violations_match_bruteforce(seed):
    net = W.random_lts(100 + seed, 3 + seed % 2, 6, 4, 2, 8, 0.25, 0.2)
    names = [f"R{r}" for r in range(net.rules.shape[0])] + \
        [f"L{l}" for l in range(net.rules.shape[0], net.n_labels)]
    mon = models.Lts(*W.random_monitor(seed, names, 4, 3))
    comp, mp, bad = models.add_monitor(net, mon, [3])
    r = oracle.explore(comp, monitor=(mp, bad))
    bf = oracle.bruteforce(comp, want_visited=True)
    assert r.levels.tolist() == bf.levels.tolist()
    words, wo, sh, wd = oracle.pack_plan(comp.n_states)
    field = (bf.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
    want = bf.visited[bad[field]]
    assert np.array_equal(r.violations, want)
    if want.shape[0]:
        # the first violating level is the smallest level index whose states
        # (oracle BFS prefix) include one
        lv = r.violation_level
        pre = oracle.explore(comp, max_levels=lv + 1, want_visited=True)
        pf = (pre.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
        assert bad[pf].any()
        if lv > 0:
            pre2 = oracle.explore(comp, max_levels=lv, want_visited=True)
            pf2 = (pre2.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
            assert not bad[pf2].any()
