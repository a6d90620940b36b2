"""CPU oracle for the exploration path of arXiv 1801.05857 -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never does: it shares
no code with it and fails loudly when its own HIP library is missing.

The C++ side (``oracle.cpp``) is a plain model of what the GPU path computes:

* ``OracleSet``: find-or-put as sequential set insertion (Sec. 4.1: insertion
  either finds the vector or stores it), backed by ``std::unordered_set``.
* ``explore``: breadth-first construction of the reachable synchronous product
  of a network of LTSs with per-level counts, transition count and deadlock
  states (Sec. 3, Fig. 1).
* ``bruteforce``: a dense-bitmap fixpoint over every vector of local states,
  used only to pin ``explore`` on tiny networks.
* ``explore_dense``: the same BFS with the visited set and the levels held
  as dense bitmaps over the product of locally reachable states and levels
  expanded by several threads, for state spaces of billions of states; it
  returns an order-independent ``digest`` of the reachable set instead of the
  set itself.
* ``pack_plan`` / ``pack``: the packing of process states into 31-bit payload
  words (Sec. 3: network data combined in 32-bit integers; Sec. 5.2: a vector
  of more than 32 bits takes several integers).

A network is any object with the attributes ``n_states`` (P ints),
``initial`` (P ints), ``trans`` (P arrays of shape (k, 3): src, label, dst),
``n_labels`` (int) and ``rules`` (R x P int32, label or -1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force: bool = True) -> str:
    """Compile ``oracle.cpp`` into ``liboracle.so`` with the host compiler."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC]
        )
        os.replace(tmp, _SO)
    return _SO


class _Result(ctypes.Structure):
    _fields_ = [
        ("words", ctypes.c_uint32),
        ("n_levels", ctypes.c_uint32),
        ("n_states", ctypes.c_uint64),
        ("n_transitions", ctypes.c_uint64),
        ("levels", ctypes.POINTER(ctypes.c_uint64)),
        ("n_deadlocks", ctypes.c_uint64),
        ("deadlocks", ctypes.POINTER(ctypes.c_uint32)),
        ("visited", ctypes.POINTER(ctypes.c_uint32)),
        ("n_violations", ctypes.c_uint64),
        ("violations", ctypes.POINTER(ctypes.c_uint32)),
        ("violation_level", ctypes.c_uint32),
    ]


class _DenseResult(ctypes.Structure):
    _fields_ = [
        ("words", ctypes.c_uint32),
        ("n_levels", ctypes.c_uint32),
        ("n_states", ctypes.c_uint64),
        ("n_transitions", ctypes.c_uint64),
        ("levels", ctypes.POINTER(ctypes.c_uint64)),
        ("n_deadlocks", ctypes.c_uint64),
        ("n_deadlocks_listed", ctypes.c_uint64),
        ("deadlocks", ctypes.POINTER(ctypes.c_uint32)),
        ("digest", ctypes.c_uint64 * 2),
        ("dead_digest", ctypes.c_uint64 * 2),
        ("index_space", ctypes.c_uint64),
        ("visited", ctypes.POINTER(ctypes.c_uint32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        lib.oracle_set_new.restype = vp
        lib.oracle_set_new.argtypes = [u32]
        lib.oracle_set_free.argtypes = [vp]
        lib.oracle_set_size.restype = u64
        lib.oracle_set_size.argtypes = [vp]
        lib.oracle_set_insert.restype = u64
        lib.oracle_set_insert.argtypes = [vp, vp, u64, vp]
        lib.oracle_set_contains.restype = i32
        lib.oracle_set_contains.argtypes = [vp, vp]
        lib.oracle_set_dump.argtypes = [vp, vp]
        lib.oracle_pack_plan.restype = i32
        lib.oracle_pack_plan.argtypes = [u32, vp, vp, vp, vp, vp]
        lib.oracle_pack.restype = i32
        lib.oracle_pack.argtypes = [u32, vp, vp, u64, vp]
        net_args = [u32, vp, vp, vp, vp, vp, vp, u32, u32, vp]
        lib.oracle_explore.restype = i32
        lib.oracle_explore.argtypes = net_args + [u64, u32, i32, ctypes.POINTER(_Result)]
        lib.oracle_explore_monitored.restype = i32
        lib.oracle_explore_monitored.argtypes = net_args + [u64, u32, i32, i32, vp, i32,
                                                            ctypes.POINTER(_Result)]
        lib.oracle_bruteforce.restype = i32
        lib.oracle_bruteforce.argtypes = net_args + [i32, ctypes.POINTER(_Result)]
        lib.oracle_result_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_successors.restype = i32
        lib.oracle_successors.argtypes = net_args + [vp, u64, vp, ctypes.POINTER(vp),
                                                     ctypes.POINTER(u64)]
        lib.oracle_free.argtypes = [vp]
        lib.oracle_digest.argtypes = [u32, vp, u64, vp]
        lib.oracle_explore_automaton.restype = i32
        lib.oracle_explore_automaton.argtypes = net_args + [u32, u32, u32, vp, vp, vp, vp, u32,
                                                            i32, i32, ctypes.POINTER(_Result)]
        lib.oracle_explore_dense.restype = i32
        lib.oracle_explore_dense.argtypes = net_args + [u32, u64, u64, i32,
                                                        ctypes.POINTER(_DenseResult)]
        lib.oracle_dense_result_free.argtypes = [ctypes.POINTER(_DenseResult)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleSet:
    """Sequential find-or-put: ``std::unordered_set`` of w-word keys."""

    def __init__(self, w: int):
        self.w = int(w)
        self._h = _load().oracle_set_new(self.w)
        if not self._h:
            raise ValueError("words per key must be 1..4")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().oracle_set_free(self._h)
            self._h = None

    def __len__(self) -> int:
        return int(_load().oracle_set_size(self._h))

    def insert(self, keys: np.ndarray) -> tuple[np.ndarray, int]:
        """Insert rows of ``keys`` (n x w uint32) in order; returns the status
        bytes (1 = new at this position, 0 = already present) and the count of
        new keys."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32).reshape(-1, self.w)
        status = np.empty(keys.shape[0], dtype=np.uint8)
        n_new = _load().oracle_set_insert(self._h, _ptr(keys), keys.shape[0], _ptr(status))
        return status, int(n_new)

    def contains(self, key) -> bool:
        k = np.ascontiguousarray(key, dtype=np.uint32).reshape(self.w)
        return bool(_load().oracle_set_contains(self._h, _ptr(k)))

    def dump(self) -> np.ndarray:
        """All keys, sorted lexicographically by (word0, word1, ...)."""
        out = np.empty((len(self), self.w), dtype=np.uint32)
        _load().oracle_set_dump(self._h, _ptr(out))
        return out


@dataclass
class OracleResult:
    words: int
    n_states: int
    n_transitions: int
    levels: np.ndarray  # uint64
    deadlocks: np.ndarray  # (n, words) uint32, sorted
    visited: np.ndarray | None  # (n_states, words) uint32, sorted
    violations: np.ndarray = None  # (n, words) uint32, sorted (safety monitor)
    violation_level: int | None = None  # first level holding a violation


def _flatten(net):
    P = len(net.n_states)
    n_states = np.ascontiguousarray(net.n_states, dtype=np.uint32)
    initial = np.ascontiguousarray(net.initial, dtype=np.uint32)
    trans = [np.asarray(t, dtype=np.uint32).reshape(-1, 3) for t in net.trans]
    n_trans = np.array([t.shape[0] for t in trans], dtype=np.uint32)
    allt = np.concatenate(trans, axis=0) if trans else np.zeros((0, 3), np.uint32)
    src = np.ascontiguousarray(allt[:, 0])
    lab = np.ascontiguousarray(allt[:, 1])
    dst = np.ascontiguousarray(allt[:, 2])
    rules = np.ascontiguousarray(net.rules, dtype=np.int32).reshape(-1, P)
    keep = (n_states, initial, n_trans, src, lab, dst, rules)
    args = [P, _ptr(n_states), _ptr(initial), _ptr(n_trans), _ptr(src), _ptr(lab), _ptr(dst),
            int(net.n_labels), rules.shape[0], _ptr(rules)]
    return args, keep


def _collect(res: _Result, want_visited: bool) -> OracleResult:
    w = res.words
    levels = np.ctypeslib.as_array(res.levels, shape=(res.n_levels,)).copy()
    if res.n_deadlocks:
        dead = np.ctypeslib.as_array(res.deadlocks, shape=(res.n_deadlocks * w,)).copy()
    else:
        dead = np.zeros(0, np.uint32)
    vis = None
    if want_visited:
        vis = np.ctypeslib.as_array(res.visited, shape=(res.n_states * w,)).copy().reshape(-1, w)
    if res.n_violations:
        viol = np.ctypeslib.as_array(res.violations, shape=(res.n_violations * w,)).copy()
    else:
        viol = np.zeros(0, np.uint32)
    vl = None if res.violation_level == 0xFFFFFFFF else int(res.violation_level)
    out = OracleResult(w, int(res.n_states), int(res.n_transitions), levels,
                       dead.reshape(-1, w), vis, viol.reshape(-1, w), vl)
    _load().oracle_result_free(ctypes.byref(res))
    return out


def explore(net, max_states: int = 0, want_visited: bool = False,
            max_levels: int = 0, monitor=None,
            stop_on_violation: bool = False) -> OracleResult:
    """Plain BFS of the synchronous product (Sec. 3).  max_levels > 0: stop
    once levels 0 .. max_levels-1 are known (a BFS prefix).  monitor =
    (process, bad) checks a safety property (Sec. 3): a state whose local
    state of that process is marked in ``bad`` (one flag per local state)
    violates it; with stop_on_violation the search ends after the first level
    that holds a violation (counted, not expanded)."""
    args, keep = _flatten(net)
    res = _Result()
    if monitor is None:
        rc = _load().oracle_explore(*args, max_states, max_levels, int(want_visited),
                                    ctypes.byref(res))
    else:
        proc, bad = monitor
        badv = np.ascontiguousarray(np.asarray(bad).astype(np.uint8))
        if badv.shape[0] != int(net.n_states[proc]):
            raise ValueError("one bad flag per local state of the monitor process")
        rc = _load().oracle_explore_monitored(*args, max_states, max_levels, int(want_visited),
                                              int(proc), _ptr(badv), int(stop_on_violation),
                                              ctypes.byref(res))
        del badv
    del keep
    if rc == -1:
        raise ValueError("invalid network")
    if rc == -2:
        raise OverflowError("more than max_states reachable states")
    return _collect(res, want_visited)


def explore_automaton(net, automaton, bad, want_visited: bool = False, max_levels: int = 0,
                      stop_on_violation: bool = False) -> OracleResult:
    """BFS of the network watched by the automaton of a negated safety
    property (Sec. 3), from the meaning of observation rather than by
    composing a network: automaton = (n_states, initial, [(src, action,
    dst)]), actions r < n_rules for rule r and n_rules + l for label l fired
    alone; ``bad`` lists its bad states.  The state packs the automaton as one
    more process after the network's."""
    args, keep = _flatten(net)
    n, init, trans = automaton
    t = np.asarray(trans, dtype=np.uint32).reshape(-1, 3)
    src, act, dst = (np.ascontiguousarray(t[:, i]) for i in range(3))
    flags = np.zeros(max(1, int(n)), dtype=np.uint8)
    flags[list(bad)] = 1
    res = _Result()
    rc = _load().oracle_explore_automaton(*args, int(n), int(init), t.shape[0], _ptr(src),
                                          _ptr(act), _ptr(dst), _ptr(flags), max_levels,
                                          int(want_visited), int(stop_on_violation),
                                          ctypes.byref(res))
    del keep
    if rc == -1:
        raise ValueError("invalid network or automaton")
    return _collect(res, want_visited)


def bruteforce(net, want_visited: bool = False) -> OracleResult:
    """Dense fixpoint enumeration for networks with prod n_p <= 2^24."""
    args, keep = _flatten(net)
    res = _Result()
    rc = _load().oracle_bruteforce(*args, int(want_visited), ctypes.byref(res))
    del keep
    if rc == -1:
        raise ValueError("invalid network")
    if rc == -2:
        raise OverflowError("product of local state counts exceeds 2^24")
    return _collect(res, want_visited)


def successors(net, states) -> tuple[np.ndarray, np.ndarray]:
    """Product successors (Sec. 3) of packed states (n x words), with
    multiplicity: (counts (n,), successors (sum(counts), words)), the
    successors of state i at rows sum(counts[:i]) ... in listing order."""
    args, keep = _flatten(net)
    words = pack_plan(net.n_states)[0]
    st = np.ascontiguousarray(states, dtype=np.uint32).reshape(-1, words)
    counts = np.zeros(st.shape[0], dtype=np.uint64)
    out = ctypes.c_void_p()
    n_out = ctypes.c_uint64()
    lib = _load()
    rc = lib.oracle_successors(*args, _ptr(st), st.shape[0], _ptr(counts), ctypes.byref(out),
                               ctypes.byref(n_out))
    del keep
    if rc != 0:
        raise ValueError("invalid network or state")
    n = int(n_out.value)
    buf = (ctypes.c_uint32 * max(1, n * words)).from_address(out.value)
    succ = np.frombuffer(buf, dtype=np.uint32, count=n * words).copy().reshape(n, words)
    lib.oracle_free(out)
    return counts, succ


def pack_plan(n_states) -> tuple[int, np.ndarray, np.ndarray, np.ndarray]:
    """(words, word_of, shift_of, width_of) of the packing rule."""
    ns = np.ascontiguousarray(n_states, dtype=np.uint32)
    P = ns.shape[0]
    wo, sh, wd = (np.zeros(P, np.uint32) for _ in range(3))
    words = np.zeros(1, np.uint32)
    if _load().oracle_pack_plan(P, _ptr(ns), _ptr(wo), _ptr(sh), _ptr(wd), _ptr(words)) != 0:
        raise ValueError("invalid process sizes")
    return int(words[0]), wo, sh, wd


def pack(n_states, local) -> np.ndarray:
    """Pack rows of local states (n x P) into rows of words."""
    ns = np.ascontiguousarray(n_states, dtype=np.uint32)
    loc = np.ascontiguousarray(local, dtype=np.uint32).reshape(-1, ns.shape[0])
    words = pack_plan(ns)[0]
    out = np.zeros((loc.shape[0], words), dtype=np.uint32)
    if _load().oracle_pack(ns.shape[0], _ptr(ns), _ptr(loc), loc.shape[0], _ptr(out)) != 0:
        raise ValueError("invalid process sizes")
    return out


def digest(states, words: int | None = None) -> tuple[int, int]:
    """Order-independent digest of a set of packed states (n x words): two
    sums modulo 2^31 - 1 of a cubic of a fixed linear form of the words.  Test
    bookkeeping for comparing sets too large to list, not part of the method."""
    st = np.ascontiguousarray(states, dtype=np.uint32)
    if words is None:
        words = st.shape[1] if st.ndim == 2 else 1
    st = st.reshape(-1, words)
    out = np.zeros(2, dtype=np.uint64)
    _load().oracle_digest(words, _ptr(st), st.shape[0], _ptr(out))
    return int(out[0]), int(out[1])


@dataclass
class DenseResult:
    words: int
    n_states: int
    n_transitions: int
    levels: np.ndarray       # uint64
    n_deadlocks: int
    deadlocks: np.ndarray | None  # (n, words) sorted; None when above the cap
    digest: tuple            # digest() of the reachable set
    dead_digest: tuple       # digest() of the deadlock set
    index_space: int         # product of the locally reachable state counts
    visited: np.ndarray | None


def explore_dense(net, threads: int = 0, max_index_space: int = 1 << 40,
                  dead_cap: int = 1 << 20, want_visited: bool = False) -> DenseResult:
    """BFS of the synchronous product (Sec. 3) over dense bitmaps, levels
    expanded by ``threads`` threads (0: one per core).  Needs three bitmaps of
    index_space bits.  Deadlocks are listed when there are at most
    ``dead_cap``; the reachable set is returned as its ``digest`` (and listed
    with want_visited)."""
    args, keep = _flatten(net)
    res = _DenseResult()
    lib = _load()
    rc = lib.oracle_explore_dense(*args, int(threads), int(max_index_space), int(dead_cap),
                                  int(want_visited), ctypes.byref(res))
    del keep
    if rc == -1:
        raise ValueError("invalid network")
    if rc == -2:
        raise OverflowError("product of locally reachable state counts exceeds the limit")
    if rc == -3:
        raise MemoryError("cannot allocate the bitmaps")
    if rc != 0:
        raise RuntimeError(f"dense exploration failed ({rc})")
    w = res.words
    levels = np.ctypeslib.as_array(res.levels, shape=(res.n_levels,)).copy()
    dead = None
    if res.n_deadlocks == res.n_deadlocks_listed:
        dead = np.zeros((0, w), np.uint32)
        if res.n_deadlocks:
            dead = np.ctypeslib.as_array(res.deadlocks, shape=(res.n_deadlocks * w,)).copy()
            dead = dead.reshape(-1, w)
    vis = None
    if want_visited:
        vis = np.ctypeslib.as_array(res.visited, shape=(res.n_states * w,)).copy().reshape(-1, w)
    out = DenseResult(w, int(res.n_states), int(res.n_transitions), levels,
                      int(res.n_deadlocks), dead, (int(res.digest[0]), int(res.digest[1])),
                      (int(res.dead_digest[0]), int(res.dead_digest[1])),
                      int(res.index_space), vis)
    lib.oracle_dense_result_free(ctypes.byref(res))
    return out
