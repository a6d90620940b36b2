"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only *produces inputs*: networks of LTSs and key streams.  It holds
none of the method's arithmetic (no packing, hashing, successor generation or
set logic), so both the GPU library and the CPU oracle can be fed from it
without sharing code with each other.

All randomness comes from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written out here from its
published definition.

Networks follow the model of Sec. 3 of the paper: a network is a list of LTSs
(states, labelled transitions, initial state) plus synchronisation rules, one
row per rule with a label per process or -1 for "does not take part".
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


# --------------------------------------------------------------------- RNG
class SplitMix64:
    """Scalar SplitMix64 stream."""

    def __init__(self, seed: int):
        self.state = seed & M64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    def below(self, k: int) -> int:
        """Uniform integer in [0, k) by multiply-high range reduction."""
        return (self.next() * k) >> 64

    def chance(self, p: float) -> bool:
        return self.next() < int(p * 2.0**64)


# ---------------------------------------------------------------- networks
@dataclass
class Network:
    """A network of LTSs with synchronisation rules (Sec. 3, Fig. 1).

    ``trans[p]`` is a (k, 3) uint32 array of (src, label, dst) for process p;
    ``rules`` is an (R, P) int32 array holding, per rule, the label each
    participating process must take, or -1 for processes that do not take part.
    """

    n_states: np.ndarray
    initial: np.ndarray
    trans: list
    n_labels: int
    rules: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_procs(self) -> int:
        return int(len(self.n_states))

    @property
    def n_transitions_local(self) -> int:
        return int(sum(t.shape[0] for t in self.trans))


def _net(n_states, initial, trans, n_labels, rules, name, **meta) -> Network:
    P = len(n_states)
    return Network(
        n_states=np.asarray(n_states, dtype=np.uint32),
        initial=np.asarray(initial, dtype=np.uint32),
        trans=[np.asarray(t, dtype=np.uint32).reshape(-1, 3) for t in trans],
        n_labels=int(n_labels),
        rules=np.asarray(rules, dtype=np.int32).reshape(-1, P),
        name=name,
        meta=dict(meta),
    )


def fig1_producer_consumers() -> Network:
    """The producer / two-consumer network of Fig. 1.

    Labels: 0 tau, 1 gen_work, 2 send, 3 rec, 4 work.  Producer: p0 -gen_work->
    p1 -send-> p0.  Consumer: c0 -rec-> c1, c1 -work-> c1, c1 -tau-> c0.  Rules
    (send, rec, _) and (send, _, rec).
    """
    producer = [(0, 1, 1), (1, 2, 0)]
    consumer = [(0, 3, 1), (1, 4, 1), (1, 0, 0)]
    rules = [[2, 3, -1], [2, -1, 3]]
    return _net([2, 2, 2], [0, 0, 0], [producer, consumer, consumer], 5, rules, "fig1")


def tiny_cycles() -> Network:
    """Four cyclic processes of 8 local states with free tau steps s -> s+1 mod 8,
    plus one rendezvous label r (an edge 0 -> 4 in every process) synchronising
    processes 0-1 and processes 2-3.  Labels: 0 tau, 1 r.  Fits one word
    (4 x 3 bits)."""
    proc = [(s, 0, (s + 1) % 8) for s in range(8)] + [(0, 1, 4)]
    rules = [[1, 1, -1, -1], [-1, -1, 1, 1]]
    return _net([8] * 4, [0] * 4, [proc] * 4, 2, rules, "tiny_cycles")


def independent_cycles(sizes) -> Network:
    """Processes that are plain tau cycles of the given sizes, no rules."""
    trans = [[(s, 0, (s + 1) % n) for s in range(n)] for n in sizes]
    return _net(list(sizes), [0] * len(sizes), trans, 1, np.zeros((0, len(sizes))),
                "cycles_" + "x".join(str(n) for n in sizes))


def token_ring(n: int) -> Network:
    """One token passed around a ring of n nodes (the Token Ring of Sec. 5.2).

    Node LTS, 5 states: A -tau-> B -tau-> C -rec-> T1 -tau-> T2 -send-> A, i.e.
    three internal transitions and two communication transitions per node.
    Rule i pairs send of node i with rec of node (i+1) mod n.  Node 0 starts
    holding the token (T1), the others in A.  Labels: 0 tau, 1 send, 2 rec.
    """
    A, B, C, T1, T2 = range(5)
    node = [(A, 0, B), (B, 0, C), (C, 2, T1), (T1, 0, T2), (T2, 1, A)]
    rules = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        rules[i, i] = 1
        rules[i, (i + 1) % n] = 2
    initial = [T1] + [A] * (n - 1)
    return _net([5] * n, initial, [node] * n, 3, rules, f"token_ring_{n}")


def random_lts(seed: int, n_procs: int, n_states, live, out_degree: int = 3,
               n_labels: int = 32, rendezvous_frac: float = 0.25, sink_prob: float = 0.0,
               name: str = "") -> Network:
    """Random network of LTSs.

    * labels 0 .. floor(rendezvous_frac * n_labels) - 1 are rendezvous labels,
      each given a seeded pair (p, q), p != q, and the rule (label@p, label@q);
      the other labels are local.
    * process p declares ``n_states[p]`` states (the encoding width) of which
      states 0 .. live[p]-1 are live; the initial state is 0.
    * every live state other than 0 is a sink with probability ``sink_prob``;
      every other live state gets ``out_degree`` transitions, each labelled with
      one of p's rendezvous labels with probability ``rendezvous_frac`` (when p
      has any) and with a uniform local label otherwise, and with a target
      uniform over the live states.
    """
    rng = SplitMix64(seed)
    ns = np.broadcast_to(np.asarray(n_states, dtype=np.int64), (n_procs,)).copy()
    lv = np.broadcast_to(np.asarray(live, dtype=np.int64), (n_procs,)).copy()
    lv = np.minimum(lv, ns)
    n_rv = int(rendezvous_frac * n_labels) if n_procs >= 2 else 0
    rules = np.full((n_rv, n_procs), -1, dtype=np.int32)
    mine = [[] for _ in range(n_procs)]
    for lab in range(n_rv):
        p = rng.below(n_procs)
        q = rng.below(n_procs - 1)
        q = q + 1 if q >= p else q
        rules[lab, p] = lab
        rules[lab, q] = lab
        mine[p].append(lab)
        mine[q].append(lab)
    trans = []
    for p in range(n_procs):
        rows = []
        for s in range(int(lv[p])):
            if s != 0 and sink_prob > 0 and rng.chance(sink_prob):
                continue
            for _ in range(out_degree):
                if mine[p] and rng.chance(rendezvous_frac):
                    lab = mine[p][rng.below(len(mine[p]))]
                else:
                    lab = n_rv + rng.below(n_labels - n_rv)
                rows.append((s, lab, rng.below(int(lv[p]))))
        trans.append(np.asarray(rows, dtype=np.uint32).reshape(-1, 3))
    return _net(ns, [0] * n_procs, trans, n_labels, rules,
                name or f"random_s{seed}_p{n_procs}", seed=seed, live=lv.tolist())


def wide_rule(n_procs: int = 6, k: int = 5) -> Network:
    """One synchronisation rule over all n_procs processes: process p has
    states 0..k, and k transitions labelled a from state 0 to states 1..k;
    states 1..k have none.  The initial state therefore has k^n_procs
    successors (one per choice of a transition in every process), all of
    them deadlocks: 1 + k^n_procs states, k^n_procs transitions, levels
    [1, k^n_procs].  A stress case for very wide per-state fan-out."""
    trans = [[(0, 0, d) for d in range(1, k + 1)] for _ in range(n_procs)]
    rules = np.zeros((1, n_procs), dtype=np.int32)
    return _net([k + 1] * n_procs, [0] * n_procs, trans, 1, rules, f"wide_rule_{n_procs}x{k}")


def degenerate_networks() -> dict:
    """Edge cases of the product semantics (Sec. 3), by name.

    lone      one process with one state and no transitions
    selfloop  one process with one state and a tau self-loop
    ones      five one-state processes, no transitions
    never     two processes whose only rule is never enabled: process 0 offers
              its label only in state 0, process 1 only in state 1
    chain     a self-looping one-state process, a tau chain 0 -> 1 -> 2 and a
              transition-less one-state process
    """
    empty_rules = lambda P: np.zeros((0, P), dtype=np.int32)
    return {
        "lone": _net([1], [0], [[]], 1, empty_rules(1), "lone"),
        "selfloop": _net([1], [0], [[(0, 0, 0)]], 1, empty_rules(1), "selfloop"),
        "ones": _net([1] * 5, [0] * 5, [[]] * 5, 1, empty_rules(5), "ones"),
        "never": _net([2, 2], [0, 0], [[(0, 1, 1)], [(1, 1, 0)]], 2, [[1, 1]], "never"),
        "chain": _net([1, 3, 1], [0, 0, 0], [[(0, 0, 0)], [(0, 0, 1), (1, 0, 2)], []], 1,
                      empty_rules(3), "chain"),
    }


def random_monitor(seed: int, actions, n_states: int = 4, n_observed: int = 4):
    """A seeded deterministic automaton over ``n_observed`` of the given action
    names (a negated safety property to add to a network): states 0 ..
    n_states-1, initial 0, one transition per (state, observed action) to a
    uniform target.  Returns (n_states, initial, [(src, action, dst)])."""
    rng = SplitMix64(seed)
    pool = list(actions)
    obs = []
    while pool and len(obs) < n_observed:
        obs.append(pool.pop(rng.below(len(pool))))
    trans = [(m, a, rng.below(n_states)) for m in range(n_states) for a in obs]
    return n_states, 0, trans


def tick_counter(n0: int, others, k: int):
    """Process 0 cycles through n0 states on action ``tick``; processes 1..
    cycle through others[i] states on ``tau``; the automaton counts ticks up
    to k and stays there (its state k is the bad one).  Returns (processes as
    (n_states, initial, trans) triples, automaton triple)."""
    procs = [(n0, 0, [(i, "tick", (i + 1) % n0) for i in range(n0)])]
    procs += [(n, 0, [(i, "tau", (i + 1) % n) for i in range(n)]) for n in others]
    mon = (k + 1, 0, [(m, "tick", min(m + 1, k)) for m in range(k + 1)])
    return procs, mon


def large_random_network(live: int = 8) -> Network:
    """The large plain-path workload: 12 processes of 64 declared local states
    (6-bit fields, so 3-word vectors), out-degree 3 with uniform targets, a
    32-label alphabet of which 25% are 2-party rendezvous between seeded
    process pairs, seed 1, sink probability 0.15.  With 8 live states per
    process 3,304,390,656 states are reachable (38 BFS levels, 90.5 G
    transitions, no deadlocks); ``live`` smaller gives the same family at
    sizes the oracle enumerates (live 3: a few hundred thousand states)."""
    return random_lts(1, 12, 64, live, 3, 32, 0.25, 0.15, name=f"large_random_l{live}")


# Table slots for the large workload: 12e9 slots of 16 bytes (192 GB), load
# factor 0.28 at its 3.3e9 states.
LARGE_TABLE_SLOTS = 12_000_000_000

# Table configuration of the large workload's exploration, the one the
# benchmark times and the full-size parity test checks: buckets of 16 words
# (four 16-byte slots, one 64-byte granule), 4-lane subgroups, one key in
# flight per subgroup, 16 hash functions.
LARGE_EXPLORE = {"bucket_words": 16, "subgroup": 4, "keys_per_subgroup": 1, "max_hashes": 16}


# ------------------------------------------------------------- key streams
MASK62 = (1 << 62) - 1


def _mix62(x: np.ndarray) -> np.ndarray:
    """A bijection of [0, 2^62): odd multiplies modulo 2^62 and xor-shifts."""
    x = x.astype(np.uint64) & np.uint64(MASK62)
    with np.errstate(over="ignore"):
        x = (x * np.uint64(0x9FB21C651E98DF25)) & np.uint64(MASK62)
        x ^= x >> np.uint64(29)
        x = (x * np.uint64(0xD6E8FEB86659FD93)) & np.uint64(MASK62)
        x ^= x >> np.uint64(32)
        x = (x * np.uint64(0x94D049BB133111EB)) & np.uint64(MASK62)
        x ^= x >> np.uint64(29)
    return x


def distinct_keys(n: int, w: int, seed: int) -> np.ndarray:
    """n distinct keys of w words, every word with bit 31 clear.

    Word 0 and word 1 come from a bijection of the counter i + seed over
    [0, 2^62), so keys are distinct for n <= 2^62 when w >= 2 (for w == 1 the
    counter itself, mixed over [0, 2^31), keeps them distinct for n <= 2^31).
    Words 2 and 3 are further mixes of the same counter.
    """
    i = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        c = (i + np.uint64(seed & MASK62)) & np.uint64(MASK62)
    out = np.empty((n, w), dtype=np.uint32)
    if w == 1:
        if n > (1 << 31):
            raise ValueError("at most 2^31 distinct one-word keys")
        x = c & np.uint64((1 << 31) - 1)
        with np.errstate(over="ignore"):
            x = (x * np.uint64(0x2545F491)) & np.uint64((1 << 31) - 1)
            x ^= x >> np.uint64(15)
            x = (x * np.uint64(0x6F4F2A35)) & np.uint64((1 << 31) - 1)
            x ^= x >> np.uint64(13)
        out[:, 0] = x.astype(np.uint32)
        return out
    x = _mix62(c)
    out[:, 0] = (x & np.uint64(0x7FFFFFFF)).astype(np.uint32)
    out[:, 1] = (x >> np.uint64(31)).astype(np.uint32)
    if w >= 3:
        y = _mix62(x ^ np.uint64(0x2AAAAAAAAAAAAAAA))
        out[:, 2] = (y & np.uint64(0x7FFFFFFF)).astype(np.uint32)
        if w == 4:
            out[:, 3] = (y >> np.uint64(31)).astype(np.uint32)
    return out


def _permute_pow2(i: np.ndarray, bits: int, seed: int) -> np.ndarray:
    """A seeded bijection of [0, 2^bits)."""
    mask = np.uint64((1 << bits) - 1)
    rng = SplitMix64(seed)
    y = i.astype(np.uint64)
    with np.errstate(over="ignore"):
        for _ in range(3):
            a = np.uint64(rng.next() | 1)
            b = np.uint64(rng.next())
            y = (y * a + b) & mask
            y ^= y >> np.uint64(max(1, bits // 2))
    return y


def permutation(n: int, seed: int) -> np.ndarray:
    """A seeded permutation of [0, n) (bijection of the next power of two,
    cycle-walked back into range)."""
    if n <= 1:
        return np.zeros(n, dtype=np.uint64)
    bits = max(1, int(n - 1).bit_length())
    y = _permute_pow2(np.arange(n, dtype=np.uint64), bits, seed)
    bad = y >= np.uint64(n)
    while bad.any():
        y[bad] = _permute_pow2(y[bad], bits, seed)
        bad = y >= np.uint64(n)
    return y


def duplicated_stream(n_distinct: int, dup: int, w: int, seed: int) -> np.ndarray:
    """A stream of n_distinct * dup keys in which each of n_distinct distinct
    keys occurs exactly ``dup`` times, in a seeded shuffled order (the key
    streams of the isolated insert experiment of Sec. 5.1)."""
    keys = distinct_keys(n_distinct, w, seed)
    n = n_distinct * dup
    order = permutation(n, seed ^ 0x5EED5EED5EED5EED)
    return keys[(order % np.uint64(n_distinct)).astype(np.int64)]


# ------------------------------------------- the same key streams, on device
def _mix62_torch(x):
    """``_mix62`` on an int64 torch tensor of values in [0, 2^62) (the
    products wrap modulo 2^64 and are masked back to 62 bits)."""
    import torch

    m = (1 << 62) - 1

    def i64(c):
        return c - (1 << 64) if c >= (1 << 63) else c

    x = x & m
    x = (x * i64(0x9FB21C651E98DF25)) & m
    x = x ^ (x >> 29)
    x = (x * i64(0xD6E8FEB86659FD93)) & m
    x = x ^ (x >> 32)
    x = (x * i64(0x94D049BB133111EB)) & m
    x = x ^ (x >> 29)
    return x


def duplicated_stream_torch(n_distinct: int, dup: int, seed: int, device, w: int = 2):
    """``duplicated_stream(n_distinct, dup, w, seed)`` generated with torch on
    ``device`` (w = 1 or 2).  Returns the (n, w) int32 key tensor and the
    int64 tensor of distinct-key indices per position."""
    import torch

    if w not in (1, 2):
        raise ValueError("one- or two-word keys")

    n = n_distinct * dup
    bits = max(1, (n - 1).bit_length())
    mask = (1 << bits) - 1
    rng = SplitMix64(seed ^ 0x5EED5EED5EED5EED)

    def i64(c):
        return c - (1 << 64) if c >= (1 << 63) else c

    consts = [(rng.next() | 1, rng.next()) for _ in range(3)]

    def permute(y):  # the seeded bijection of [0, 2^bits) of permutation()
        for a, b in consts:
            y = (y * i64(a) + i64(b)) & mask
            y = y ^ (y >> max(1, bits // 2))
        return y

    y = permute(torch.arange(n, dtype=torch.int64, device=device))
    bad = y >= n
    while bool(bad.any()):  # cycle-walk back into [0, n)
        y[bad] = permute(y[bad])
        bad = y >= n
    idx = y % n_distinct
    c = (idx + (seed & MASK62)) & MASK62
    if w == 1:
        m31 = (1 << 31) - 1
        x = c & m31
        x = (x * 0x2545F491) & m31
        x = x ^ (x >> 15)
        x = (x * 0x6F4F2A35) & m31
        x = x ^ (x >> 13)
        return x.to(torch.int32).reshape(n, 1), idx
    x = _mix62_torch(c)
    keys = torch.empty((n, 2), dtype=torch.int32, device=device)
    keys[:, 0] = (x & 0x7FFFFFFF).to(torch.int32)
    keys[:, 1] = (x >> 31).to(torch.int32)
    return keys, idx


# ------------------------------------------------ batches of uneven networks
def batch_networks(n: int, seed: int, log10_lo: float = 3.0, log10_hi: float = 7.0,
                   procs=(3, 10), states=(4, 64), out_degree: int = 3):
    """n random networks for batched exploration, with uneven sizes.

    Instance i: P ~ U{procs}, declared states n_p ~ U{states} per process, a
    target T ~ log-uniform [10^lo, 10^hi], and live-state counts m_p (2 <=
    m_p <= n_p) chosen so that prod m_p is close to 4T.  Every reachable local
    state is live, so prod m_p bounds the reachable set; it is returned as the
    instance's capacity.  Returns (networks, capacities).
    """
    import math

    rng = SplitMix64(seed)
    nets, caps = [], []
    for i in range(n):
        P = procs[0] + rng.below(procs[1] - procs[0] + 1)
        ns = [states[0] + rng.below(states[1] - states[0] + 1) for _ in range(P)]
        u = rng.next() / 2.0**64
        target = 10 ** (log10_lo + (log10_hi - log10_lo) * u)
        want = 4.0 * target
        m = [2] * P
        # raise the live counts round-robin while the product stays below 4T
        grew = True
        while grew:
            grew = False
            for p in range(P):
                if m[p] < ns[p] and math.prod(m) / m[p] * (m[p] + 1) <= want:
                    m[p] += 1
                    grew = True
        nets.append(random_lts(seed * 100003 + i, P, ns, m, out_degree, 32, 0.25, 0.05,
                               name=f"batch_{seed}_{i}"))
        caps.append(int(math.prod(m)))
    return nets, caps


# --------------------------------------------------- served exploration requests
def served_networks(n: int, seed: int, log10_lo: float = 4.0, log10_hi: float = 8.0,
                    out_degree: int = 3):
    """n random networks for the served workload, sizes and vector widths
    decoupled.

    Request i: a target T ~ log-uniform [10^lo, 10^hi] and a width w ~ U{1..4}
    words; P processes of 64 declared states (6-bit fields, five per word),
    P ~ U{5(w-1)+1 .. 5w} raised until 64^P >= 2T; live counts m_p
    (1 <= m_p <= 64) raised round-robin while prod m_p <= 2T (a third to all
    of the product is reachable, so reachable sizes centre on T).  Every
    reachable local state is live, so prod m_p bounds the reachable set; it
    is the request's declared bound.  Returns (networks, targets, bounds)."""
    import math

    rng = SplitMix64(seed)
    nets, targets, bounds = [], [], []
    for i in range(n):
        u = rng.next() / 2.0**64
        target = 10 ** (log10_lo + (log10_hi - log10_lo) * u)
        w = 1 + rng.below(4)
        P = 5 * (w - 1) + 1 + rng.below(5)
        while 64 ** P < 2 * target and P < 5 * w:
            P += 1
        want = 2.0 * target
        m = [1] * P
        grew = True
        while grew:
            grew = False
            for p in range(P):
                if m[p] < 64 and math.prod(m) / m[p] * (m[p] + 1) <= want:
                    m[p] += 1
                    grew = True
        nets.append(random_lts(seed * 1000003 + i, P, 64, m, out_degree, 32, 0.25, 0.05,
                               name=f"served_{seed}_{i}"))
        targets.append(int(target))
        bounds.append(int(math.prod(m)))
    return nets, targets, bounds
