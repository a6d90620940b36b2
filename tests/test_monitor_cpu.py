"""Safety monitors (Sec. 3: the negation of a safety property is an automaton
added to the network; reaching one of its bad states is a violation).

The oracle watches the network with the automaton directly
(``oracle.explore_automaton``: every network action moves the automaton along
its transitions on that action).  It is pinned here to closed forms, hand-
derived cases and the brute-force fixpoint; the library's composition
(``gx_network_add_monitor``, host code) is checked against it: the oracle's
plain search of the composed network gives the same results."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W
from paper_1801_05857_amd import models


def _tick_raw(n0, others, k):
    """The tick-counter family as a raw network plus an automaton over action
    numbers: process 0 fires label 0 ("tick") alone, the others label 1
    ("tau"); no rules, so tick is action 0 + 0 = 0."""
    procs, mon = W.tick_counter(n0, others, k)
    trans = [[(s, 0 if a == "tick" else 1, d) for s, a, d in pr[2]] for pr in procs]
    net = W.Network(np.array([pr[0] for pr in procs], np.uint32),
                    np.zeros(len(procs), np.uint32),
                    [np.asarray(t, np.uint32).reshape(-1, 3) for t in trans], 2,
                    np.zeros((0, len(procs)), np.int32))
    aut = (mon[0], mon[1], [(s, 0, d) for s, _, d in mon[2]])
    return net, aut


def _tick_levels(n0, others, k):
    hist = np.ones(k + n0, dtype=np.int64)
    for n in others:
        hist = np.convolve(hist, np.ones(n, dtype=np.int64))
    return hist


@pytest.mark.parametrize("n0,others,k", [(5, [3, 4], 7), (4, [2], 2), (3, [5], 0),
                                         (6, [], 9), (2, [2, 2, 3], 1)])
def test_tick_counter_closed_form(n0, others, k):
    # (process 0, automaton) reach the chain (m ticks, m mod n0) for m < k and
    # then every (k, p0): k + n0 states at distances 0 .. k + n0 - 1; the other
    # cycles are independent, so levels are the convolution of the distance
    # histograms, and the violations are the n0 * prod(others) states with
    # the automaton at k, first reached at distance k
    net, aut = _tick_raw(n0, others, k)
    hist = _tick_levels(n0, others, k)
    prod = int(np.prod(others)) if others else 1
    r = oracle.explore_automaton(net, aut, [k])
    assert r.levels.tolist() == hist.tolist()
    assert r.n_states == (k + n0) * prod
    assert r.violations.shape[0] == n0 * prod
    assert r.violation_level == k
    # stopping at the first violation: levels 0..k, one violating state
    s = oracle.explore_automaton(net, aut, [k], stop_on_violation=True)
    assert s.levels.tolist() == hist[:k + 1].tolist()
    assert s.n_states == int(hist[:k + 1].sum())
    assert s.violations.shape[0] == 1 and s.violation_level == k


@pytest.mark.parametrize("n,k", [(5, 3), (4, 0), (3, 8)])
def test_observed_rule_closed_form(n, k):
    # two n-cycles that step together through one rule (action 0): n states on
    # one diagonal; an automaton counting the rule up to k: the same chain as
    # the tick counter with no other process
    step = np.array([(i, 0, (i + 1) % n) for i in range(n)], np.uint32)
    net = W.Network(np.array([n, n], np.uint32), np.zeros(2, np.uint32), [step, step], 1,
                    np.array([[0, 0]], np.int32))
    aut = (k + 1, 0, [(m, 0, min(m + 1, k)) for m in range(k + 1)])
    r = oracle.explore_automaton(net, aut, [k])
    assert r.levels.tolist() == [1] * (k + n)
    assert r.n_transitions == k + n
    assert r.violations.shape[0] == n and r.violation_level == k


def test_nondeterministic_automaton_by_hand():
    # one state with a self-loop on label 0 (action 0, no rules); the automaton
    # leaves state 0 on that action for 1 or 2 and then stays: states (0,0),
    # (0,1), (0,2); transitions 2 + 1 + 1; state 2 is bad
    net = W.Network(np.array([1], np.uint32), np.zeros(1, np.uint32),
                    [np.array([[0, 0, 0]], np.uint32)], 1, np.zeros((0, 1), np.int32))
    aut = (3, 0, [(0, 0, 1), (0, 0, 2), (1, 0, 1), (2, 0, 2)])
    r = oracle.explore_automaton(net, aut, [2], want_visited=True)
    assert r.levels.tolist() == [1, 2] and r.n_transitions == 4
    assert r.violations.tolist() == [[0 | (2 << 1)]]  # 1-bit field, then 2 bits
    assert r.violation_level == 1
    # an automaton with no transition on the action in state 1 stays there
    aut = (2, 0, [(0, 0, 1)])
    r = oracle.explore_automaton(net, aut, [1])
    assert r.levels.tolist() == [1, 1] and r.n_transitions == 2


def test_automaton_that_never_moves_changes_nothing():
    net = W.random_lts(17, 4, 8, 4, 3, 16, 0.25, 0.2)
    R = net.rules.shape[0]
    acts = list(range(R + net.n_labels))
    a = oracle.explore(net)
    for aut in [(1, 0, [(0, x, 0) for x in acts[::3]]), (1, 0, [])]:
        b = oracle.explore_automaton(net, aut, [])
        assert a.levels.tolist() == b.levels.tolist()
        assert a.n_transitions == b.n_transitions
        assert b.violations.shape[0] == 0 and b.violation_level is None


def _random_case(seed, P=None):
    P = P or 3 + seed % 2
    net = W.random_lts(100 + seed, P, 6, 4, 2, 8, 0.25, 0.2)
    acts = list(range(net.rules.shape[0] + net.n_labels))
    aut = W.random_monitor(seed, acts, 4, 3)
    return net, aut


@pytest.mark.parametrize("seed", range(8))
def test_violations_match_bruteforce(seed):
    # the brute-force fixpoint runs over the composed network (the automaton
    # as one more process); the violations are its reachable states whose
    # automaton field is bad, the first violating level the first BFS prefix
    # holding one
    net, aut = _random_case(seed)
    comp, mp, bad = gx.add_monitor(net, aut, [3])
    r = oracle.explore_automaton(net, aut, [3])
    bf = oracle.bruteforce(comp, want_visited=True)
    assert r.levels.tolist() == bf.levels.tolist()
    assert r.n_transitions == bf.n_transitions
    words, wo, sh, wd = oracle.pack_plan(comp.n_states)
    field = (bf.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
    want = bf.visited[bad[field]]
    assert np.array_equal(r.violations, want)
    if want.shape[0]:
        lv = r.violation_level
        pre = oracle.explore_automaton(net, aut, [3], max_levels=lv + 1, want_visited=True)
        pf = (pre.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
        assert bad[pf].any()
        if lv > 0:
            pre2 = oracle.explore_automaton(net, aut, [3], max_levels=lv, want_visited=True)
            pf2 = (pre2.visited[:, wo[mp]] >> sh[mp]) & ((1 << int(wd[mp])) - 1)
            assert not bad[pf2].any()


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("stop", [False, True])
def test_library_composition_equals_oracle(seed, stop):
    """gx_network_add_monitor (host code of the library) composes the network
    whose plain search gives what the oracle's observation semantics gives."""
    net, aut = _random_case(seed, P=3 + seed % 5)
    comp, mp, bad = gx.add_monitor(net, aut, [3])
    assert mp == net.n_procs and len(comp.n_states) == net.n_procs + 1
    a = oracle.explore_automaton(net, aut, [3], want_visited=True, stop_on_violation=stop)
    b = oracle.explore(comp, monitor=(mp, bad), want_visited=True, stop_on_violation=stop)
    assert a.levels.tolist() == b.levels.tolist()
    assert a.n_transitions == b.n_transitions
    assert np.array_equal(a.visited, b.visited)
    assert np.array_equal(a.deadlocks, b.deadlocks)
    assert np.array_equal(a.violations, b.violations)
    assert a.violation_level == b.violation_level


def test_library_composition_rejects_bad_automata():
    net = W.random_lts(3, 3, 6, 4, 2, 8, 0.25, 0.2)
    n_act = net.rules.shape[0] + net.n_labels
    with pytest.raises(gx.GxError):
        gx.add_monitor(net, (2, 0, [(0, n_act, 1)]), [1])  # action out of range
    with pytest.raises(gx.GxError):
        gx.add_monitor(net, (2, 2, []), [1])  # initial state out of range
    with pytest.raises(gx.GxError):
        gx.add_monitor(net, (2, 0, [(0, 0, 5)]), [1])  # target out of range


def test_names_map_to_actions():
    """models.add_monitor (names) equals the action-number form: the tick
    counter written as .aut files and a par network."""
    procs, mon = W.tick_counter(5, [3, 4], 7)
    files = {f"p{i}.aut": models.write_aut(*pr) for i, pr in enumerate(procs)}
    par = "par using in " + " || ".join(f'"p{i}.aut"' for i in range(len(procs))) + " end par"
    comp, mp, bad = models.add_monitor(models.parse_par(par, files), models.Lts(*mon), [7])
    r = oracle.explore(comp, monitor=(mp, bad))
    net, aut = _tick_raw(5, [3, 4], 7)
    s = oracle.explore_automaton(net, aut, [7])
    assert r.levels.tolist() == s.levels.tolist()
    assert r.violations.shape[0] == s.violations.shape[0] and r.violation_level == 7
