"""Loaders for the input formats of the paper's models (Sec. 3, Fig. 1).

* Aldebaran ``.aut`` files describe one LTS: a header ``des (initial,
  n_transitions, n_states)`` followed by one ``(src, "label", dst)`` line per
  transition.
* A network is written in the EXP.OPEN ``par`` syntax of Fig. 1:

      par using
          send * rec * _ -> trans,
          send * _ * rec -> trans
      in
          "producer.aut" || "consumer.aut" || "consumer.aut"
      end par

  Each synchronisation vector lists, per process, the label it takes or ``_``
  when it does not take part (the result label after ``->`` is kept only as a
  name).  Labels named by a vector at a process's position fire only through
  vectors; every other label of that process fires alone.

The result is a plain network description (states, initial state and
(src, label, dst) transitions per process, label count, rule matrix) that the
C ABI (``gx_network``) takes.  Labels are numbered over the whole network, in
order of first appearance; ``i`` (the internal action of Aldebaran files) and
``tau`` are ordinary labels here.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Lts:
    n_states: int
    initial: int
    trans: list  # (src, label name, dst)


@dataclass
class LoadedNetwork:
    n_states: np.ndarray
    initial: np.ndarray
    trans: list          # per process: (k, 3) uint32 array of (src, label id, dst)
    n_labels: int
    rules: np.ndarray    # (R, P) int32: label id per process or -1
    labels: list = field(default_factory=list)        # label id -> name
    rule_names: list = field(default_factory=list)    # result label of each vector


_HEADER = re.compile(r"^\s*des\s*\(\s*(\d+)\s*,\s*(\d+)\s*,\s*(\d+)\s*\)\s*$")
_EDGE = re.compile(r'^\s*\(\s*(\d+)\s*,\s*("(?:[^"\\]|\\.)*"|[^,()]+?)\s*,\s*(\d+)\s*\)\s*$')


def parse_aut(text: str) -> Lts:
    """Parse the text of an Aldebaran file."""
    lines = [ln for ln in text.splitlines() if ln.strip()]
    if not lines:
        raise ValueError("empty .aut text")
    m = _HEADER.match(lines[0])
    if not m:
        raise ValueError(f"bad .aut header: {lines[0]!r}")
    initial, n_trans, n_states = (int(x) for x in m.groups())
    trans = []
    for ln in lines[1:]:
        e = _EDGE.match(ln)
        if not e:
            raise ValueError(f"bad .aut transition line: {ln!r}")
        src, lab, dst = int(e.group(1)), e.group(2).strip(), int(e.group(3))
        if lab.startswith('"'):
            lab = lab[1:-1]
        if src >= n_states or dst >= n_states:
            raise ValueError(f"state out of range in {ln!r}")
        trans.append((src, lab, dst))
    if len(trans) != n_trans:
        raise ValueError(f"header announces {n_trans} transitions, file has {len(trans)}")
    if initial >= n_states:
        raise ValueError("initial state out of range")
    return Lts(n_states, initial, trans)


def _split_top(text: str, sep: str) -> list:
    return [x.strip() for x in text.split(sep)]


def parse_par(text: str, files: dict) -> LoadedNetwork:
    """Parse an EXP.OPEN ``par using ... in ... end par`` network.

    ``files`` maps each quoted file name to the text of that ``.aut`` file.
    """
    src = re.sub(r"\(\*.*?\*\)", " ", text, flags=re.S)  # EXP comments
    m = re.search(r"\bpar\s+using\b(.*?)\bin\b(.*?)\bend\s+par\b", src, flags=re.S)
    if not m:
        raise ValueError("expected 'par using <vectors> in <processes> end par'")
    vec_text, proc_text = m.group(1), m.group(2)
    names = re.findall(r'"([^"]+)"', proc_text)
    if not names or len(names) != len(_split_top(proc_text.strip(), "||")):
        raise ValueError("processes must be quoted .aut file names separated by '||'")
    ltss = []
    for nm in names:
        if nm not in files:
            raise ValueError(f"no text given for {nm!r}")
        ltss.append(parse_aut(files[nm]))
    P = len(ltss)
    labels: list = []
    index: dict = {}

    def lid(name: str) -> int:
        if name not in index:
            index[name] = len(labels)
            labels.append(name)
        return index[name]

    rules, rule_names = [], []
    for vec in [v for v in _split_top(vec_text, ",") if v]:
        if "->" not in vec:
            raise ValueError(f"vector without '->': {vec!r}")
        lhs, res = (x.strip() for x in vec.split("->", 1))
        parts = _split_top(lhs, "*")
        if len(parts) != P:
            raise ValueError(f"vector {vec!r} has {len(parts)} components for {P} processes")
        row = [-1 if p == "_" else lid(p) for p in parts]
        if all(x < 0 for x in row):
            raise ValueError(f"vector {vec!r} has no participant")
        rules.append(row)
        rule_names.append(res)
    trans = []
    for lts in ltss:
        rows = [(s, lid(lab), d) for s, lab, d in lts.trans]
        trans.append(np.asarray(rows, dtype=np.uint32).reshape(-1, 3))
    return LoadedNetwork(
        n_states=np.array([l.n_states for l in ltss], dtype=np.uint32),
        initial=np.array([l.initial for l in ltss], dtype=np.uint32),
        trans=trans,
        n_labels=max(1, len(labels)),
        rules=np.asarray(rules, dtype=np.int32).reshape(-1, P),
        labels=labels,
        rule_names=rule_names,
    )


def add_monitor(net, monitor: Lts, bad) -> tuple:
    """Add the automaton of a negated safety property to a network (Sec. 3).

    The automaton observes actions by name: the result label of a
    synchronisation vector, or the label of a transition that a process fires
    alone.  Every observed action then takes the automaton along: a vector
    whose result it observes gains the automaton as a participant, and a
    label that process p fires alone becomes a vector of p and the automaton.
    Actions the automaton does not observe fire as before.  Readings: an
    observed action that the automaton does not specify in some state leaves
    it in that state (the automaton is completed with self-loops, so it
    never blocks the network), and actions it names but the network never
    performs are dropped.

    ``net`` needs ``n_states``, ``initial``, ``trans``, ``n_labels`` and
    ``rules``; its ``labels`` and ``rule_names``, when present, name actions
    (otherwise labels are ``L<id>`` and vectors ``R<index>``).  ``bad`` lists
    the automaton's bad states.  Returns (network with the automaton as its
    last process, that process's index, per-state bad flags).
    """
    P = len(net.n_states)
    rules = np.asarray(net.rules, dtype=np.int32).reshape(-1, P)
    labels = list(getattr(net, "labels", None) or [f"L{i}" for i in range(net.n_labels)])
    rule_names = list(getattr(net, "rule_names", None) or
                      [f"R{r}" for r in range(rules.shape[0])])
    labels = labels + [f"L{i}" for i in range(len(labels), net.n_labels)]
    index = {nm: i for i, nm in enumerate(labels)}

    def lid(name: str) -> int:
        if name not in index:
            index[name] = len(labels)
            labels.append(name)
        return index[name]

    alphabet = {lab for _, lab, _ in monitor.trans}
    performed = set()
    new_rules, names = [], []
    for r in range(rules.shape[0]):
        nm = rule_names[r]
        obs = nm in alphabet
        if obs:
            performed.add(nm)
        new_rules.append(list(rules[r]) + [lid(nm) if obs else -1])
        names.append(nm)
    for p in range(P):
        governed = set(int(x) for x in rules[:, p] if x >= 0)
        used = set(int(x) for x in np.asarray(net.trans[p], dtype=np.int64).reshape(-1, 3)[:, 1])
        for lab in sorted(used - governed):
            nm = labels[lab]
            if nm in alphabet:
                performed.add(nm)
                row = [-1] * (P + 1)
                row[p], row[P] = lab, lid(nm)
                new_rules.append(row)
                names.append(nm)
    have = {(s_, a) for s_, a, _ in monitor.trans}
    mt = [(s_, lid(a), d) for s_, a, d in monitor.trans if a in performed]
    for m in range(monitor.n_states):
        for a in sorted(performed):
            if (m, a) not in have:
                mt.append((m, lid(a), m))
    bad_flags = np.zeros(monitor.n_states, dtype=bool)
    bad_flags[list(bad)] = True
    composed = LoadedNetwork(
        n_states=np.append(np.asarray(net.n_states, np.uint32), np.uint32(monitor.n_states)),
        initial=np.append(np.asarray(net.initial, np.uint32), np.uint32(monitor.initial)),
        trans=[np.asarray(t, dtype=np.uint32).reshape(-1, 3) for t in net.trans] +
              [np.asarray(mt, dtype=np.uint32).reshape(-1, 3)],
        n_labels=max(1, len(labels)),
        rules=np.asarray(new_rules, dtype=np.int32).reshape(-1, P + 1),
        labels=labels,
        rule_names=names,
    )
    return composed, P, bad_flags


def write_aut(n_states: int, initial: int, trans) -> str:
    """Text of an Aldebaran file for (src, label name, dst) transitions."""
    out = [f"des ({initial}, {len(trans)}, {n_states})"]
    out += [f'({s}, "{lab}", {d})' for s, lab, d in trans]
    return "\n".join(out) + "\n"
