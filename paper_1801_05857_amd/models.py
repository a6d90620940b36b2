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
    """Add the automaton of a negated safety property, given with action
    names, to a network (Sec. 3), through gx_network_add_monitor.

    The automaton observes actions by name: the result label of a
    synchronisation vector (``rule_names``), or a label (``labels``) that a
    process fires alone; a name that is both stands for both actions.  Names
    become the action numbers of gx_monitor (rule r; n_rules + l for label l
    fired alone) and the library composes the network (see gx.h).  ``net``
    needs ``n_states``, ``initial``, ``trans``, ``n_labels`` and ``rules``;
    without ``labels`` / ``rule_names`` labels are named ``L<id>`` and vectors
    ``R<index>``.  ``bad`` lists the automaton's bad states.  Returns (network
    with the automaton as its last process, that process's index, per-state
    bad flags)."""
    from . import add_monitor as gx_add_monitor

    P = len(net.n_states)
    rules = np.asarray(net.rules, dtype=np.int32).reshape(-1, P)
    R = rules.shape[0]
    labels = list(getattr(net, "labels", None) or [f"L{i}" for i in range(net.n_labels)])
    labels = labels + [f"L{i}" for i in range(len(labels), net.n_labels)]
    rule_names = list(getattr(net, "rule_names", None) or [f"R{r}" for r in range(R)])
    trans = []
    for src, name, dst in monitor.trans:
        trans += [(src, r, dst) for r in range(R) if rule_names[r] == name]
        trans += [(src, R + l, dst) for l in range(net.n_labels) if labels[l] == name]
    comp, mp, flags = gx_add_monitor(net, (monitor.n_states, monitor.initial, trans), bad)
    return comp, mp, flags


def write_aut(n_states: int, initial: int, trans) -> str:
    """Text of an Aldebaran file for (src, label name, dst) transitions."""
    out = [f"des ({initial}, {len(trans)}, {n_states})"]
    out += [f'({s}, "{lab}", {d})' for s, lab, d in trans]
    return "\n".join(out) + "\n"
