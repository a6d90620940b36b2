"""Python binding of ``libgx.so`` (declared in include/gx.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors (their ``data_ptr()``), streams are
torch streams (their ``cuda_stream`` handle); when no stream is given the
current torch stream is used, so work is ordered with the caller's torch ops.

There is no fallback: if ``libgx.so`` is missing every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgx.so")

# status codes (gx_status)
GX_OK, GX_EINVAL, GX_ENOMEM, GX_ETABLEFULL, GX_EDEVICE, GX_EBUSY, GX_ECANCELED = (
    0, -1, -2, -3, -4, -5, -6)
# per-key status bytes
GX_SEEN, GX_NEW, GX_FULL, GX_INVALID = 0, 1, 2, 3
EMPTY_WORD = 0xFFFFFFFF

EXPORTED = [
    "gx_table_create", "gx_table_destroy", "gx_table_clear", "gx_find_or_put",
    "gx_table_get_info", "gx_table_stats", "gx_table_dump", "gx_table_read_raw",
    "gx_table_copy_raw",
    "gx_hash_bucket", "gx_network_words", "gx_network_pack", "gx_explore",
    "gx_explore_result_free", "gx_status_str", "gx_gather_probe",
    "gx_batch_create", "gx_batch_run", "gx_batch_results", "gx_batch_instance_config",
    "gx_batch_destroy", "gx_explore_batch", "gx_autotune", "gx_autotune_capacity",
    "gx_server_create", "gx_server_submit", "gx_server_poll", "gx_server_get_stats",
    "gx_server_destroy", "gx_network_add_monitor", "gx_monitored_network_free",
    "gx_explore_noalloc", "gx_claim_probe",
]


class GxError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_str(code)} ({code})")


class _TableOpts(ctypes.Structure):
    _fields_ = [("hash_seed", ctypes.c_uint64), ("max_hashes", ctypes.c_uint32),
                ("subgroup", ctypes.c_uint32), ("keys_per_subgroup", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _TableInfo(ctypes.Structure):
    _fields_ = [("words_per_state", ctypes.c_uint32), ("slot_words", ctypes.c_uint32),
                ("bucket_words", ctypes.c_uint32), ("subgroup", ctypes.c_uint32),
                ("keys_per_subgroup", ctypes.c_uint32), ("max_hashes", ctypes.c_uint32),
                ("n_buckets", ctypes.c_uint64), ("n_slots", ctypes.c_uint64),
                ("hash_seed", ctypes.c_uint64), ("bytes", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("stored", ctypes.c_uint64), ("lookups", ctypes.c_uint64),
                ("probes", ctypes.c_uint64), ("full", ctypes.c_uint64),
                ("invalid", ctypes.c_uint64), ("max_hash_index", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _Lts(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint32), ("initial", ctypes.c_uint32),
                ("n_trans", ctypes.c_uint32), ("src", ctypes.c_void_p),
                ("label", ctypes.c_void_p), ("dst", ctypes.c_void_p)]


class _Network(ctypes.Structure):
    _fields_ = [("n_procs", ctypes.c_uint32), ("procs", ctypes.POINTER(_Lts)),
                ("n_labels", ctypes.c_uint32), ("n_rules", ctypes.c_uint32),
                ("rules", ctypes.c_void_p)]


class _ExploreOpts(ctypes.Structure):
    _fields_ = [("frontier_capacity", ctypes.c_uint64), ("deadlock_capacity", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("local_dedup", ctypes.c_uint32),
                ("monitor_proc", ctypes.c_uint32), ("stop_on_violation", ctypes.c_uint32),
                ("slice_states", ctypes.c_uint32), ("monitor_bad", ctypes.c_void_p)]


class _ExploreResult(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint64), ("n_transitions", ctypes.c_uint64),
                ("words_per_state", ctypes.c_uint32), ("n_levels", ctypes.c_uint32),
                # (library-owned arrays as plain addresses: copied out by _take_result)
                ("level_counts", ctypes.c_void_p),
                ("n_deadlocks", ctypes.c_uint64), ("deadlocks", ctypes.c_void_p),
                ("local_duplicates", ctypes.c_uint64),
                ("n_violations", ctypes.c_uint64), ("violations", ctypes.c_void_p),
                ("violation_level", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("states", ctypes.c_void_p)]


class _Monitor(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint32), ("initial", ctypes.c_uint32),
                ("n_trans", ctypes.c_uint32), ("src", ctypes.c_void_p),
                ("action", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("bad", ctypes.c_void_p)]


class _MonitoredNetwork(ctypes.Structure):
    _fields_ = [("net", _Network), ("monitor_proc", ctypes.c_uint32),
                ("monitor_bad", ctypes.POINTER(ctypes.c_uint8)), ("owner", ctypes.c_void_p)]


class _ExploreSummary(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint64), ("n_transitions", ctypes.c_uint64),
                ("n_levels", ctypes.c_uint32), ("words_per_state", ctypes.c_uint32),
                ("n_deadlocks", ctypes.c_uint64)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_void_p), ("hash_seed", ctypes.c_uint64),
                ("max_hashes", ctypes.c_uint32), ("bucket_words", ctypes.c_uint32),
                ("subgroup", ctypes.c_uint32), ("keys_per_subgroup", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("max_levels", ctypes.c_uint32),
                ("deadlock_capacity", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
                ("keep_states", ctypes.c_uint32), ("persistent", ctypes.c_uint32)]


class _TuneInfo(ctypes.Structure):
    _fields_ = [("bucket_words", ctypes.c_uint32), ("subgroup", ctypes.c_uint32),
                ("keys_per_subgroup", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("ns_per_key", ctypes.c_double), ("ns_per_key_default", ctypes.c_double),
                ("ns_per_key_runner_up", ctypes.c_double), ("table_slots", ctypes.c_uint64),
                ("size_class", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("max_hashes", ctypes.c_uint32), ("load_factor", ctypes.c_double),
                ("hash_seed", ctypes.c_uint64), ("bucket_words", ctypes.c_uint32),
                ("subgroup", ctypes.c_uint32), ("keys_per_subgroup", ctypes.c_uint32),
                ("keep_states", ctypes.c_uint32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "failed", "retried", "steps", "active_peak", "reserved_peak",
        "states", "reserved_now", "pooled_bytes", "waiting")]


_lib_handle = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                "g.build()'` (or paper_1801_05857_amd/build.py); there is no fallback path")
        # torch's HIP runtime is loaded first, so that the library binds to
        # the same one: loaded the other way round, torch finds no GPU once
        # the library has touched the device
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        st, vp, u32, u64 = ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.gx_table_create.restype = st
        L.gx_table_create.argtypes = [u32, u32, u64, ctypes.POINTER(_TableOpts),
                                      ctypes.POINTER(vp)]
        L.gx_table_destroy.restype = st
        L.gx_table_destroy.argtypes = [vp]
        L.gx_table_clear.restype = st
        L.gx_table_clear.argtypes = [vp, vp]
        L.gx_find_or_put.restype = st
        L.gx_find_or_put.argtypes = [vp, vp, u64, vp, vp, vp]
        L.gx_table_get_info.restype = st
        L.gx_table_get_info.argtypes = [vp, ctypes.POINTER(_TableInfo)]
        L.gx_table_stats.restype = st
        L.gx_table_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.gx_table_dump.restype = st
        L.gx_table_dump.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
        L.gx_table_read_raw.restype = st
        L.gx_table_read_raw.argtypes = [vp, vp, u64, u64]
        L.gx_explore_noalloc.restype = st
        L.gx_explore_noalloc.argtypes = [ctypes.POINTER(_Network), vp,
                                         ctypes.POINTER(_ExploreOpts), vp, u32, vp, u64,
                                         ctypes.POINTER(_ExploreSummary)]
        L.gx_network_add_monitor.restype = st
        L.gx_network_add_monitor.argtypes = [ctypes.POINTER(_Network), ctypes.POINTER(_Monitor),
                                             ctypes.POINTER(_MonitoredNetwork)]
        L.gx_monitored_network_free.restype = None
        L.gx_monitored_network_free.argtypes = [ctypes.POINTER(_MonitoredNetwork)]
        L.gx_table_copy_raw.restype = st
        L.gx_table_copy_raw.argtypes = [vp, vp, u64, u64, vp]
        L.gx_hash_bucket.restype = st
        L.gx_hash_bucket.argtypes = [vp, u32, u64, u32, u64, ctypes.POINTER(u64)]
        L.gx_network_words.restype = st
        L.gx_network_words.argtypes = [ctypes.POINTER(_Network), ctypes.POINTER(u32)]
        L.gx_network_pack.restype = st
        L.gx_network_pack.argtypes = [ctypes.POINTER(_Network), vp, u64, vp]
        L.gx_explore.restype = st
        L.gx_explore.argtypes = [ctypes.POINTER(_Network), vp, ctypes.POINTER(_ExploreOpts),
                                 ctypes.POINTER(_ExploreResult)]
        L.gx_explore_result_free.restype = None
        L.gx_explore_result_free.argtypes = [ctypes.POINTER(_ExploreResult)]
        L.gx_status_str.restype = ctypes.c_char_p
        L.gx_status_str.argtypes = [st]
        L.gx_claim_probe.restype = st
        L.gx_claim_probe.argtypes = [vp, u64, u32, u64, u64, vp, vp]
        L.gx_gather_probe.restype = st
        L.gx_gather_probe.argtypes = [vp, u64, u32, u64, u64, vp, vp]
        L.gx_batch_create.restype = st
        L.gx_batch_create.argtypes = [vp, u32, ctypes.POINTER(_BatchOpts), ctypes.POINTER(vp)]
        L.gx_batch_run.restype = st
        L.gx_batch_run.argtypes = [vp, vp]
        L.gx_batch_results.restype = st
        L.gx_batch_results.argtypes = [vp, vp, vp]
        L.gx_batch_instance_config.restype = st
        L.gx_batch_instance_config.argtypes = [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                               ctypes.POINTER(u32)]
        L.gx_batch_destroy.restype = st
        L.gx_batch_destroy.argtypes = [vp]
        L.gx_explore_batch.restype = st
        L.gx_explore_batch.argtypes = [vp, u32, ctypes.POINTER(_BatchOpts), vp, vp]
        L.gx_autotune_capacity.restype = st
        L.gx_autotune_capacity.argtypes = [u32, ctypes.c_double, u64, ctypes.POINTER(_TuneInfo)]
        L.gx_autotune.restype = st
        L.gx_autotune.argtypes = [u32, ctypes.c_double, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                  ctypes.POINTER(u32)]
        L.gx_server_create.restype = st
        L.gx_server_create.argtypes = [ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)]
        L.gx_server_submit.restype = st
        L.gx_server_submit.argtypes = [vp, ctypes.POINTER(_Network), u64, ctypes.POINTER(u64)]
        L.gx_server_poll.restype = st
        L.gx_server_poll.argtypes = [vp, u64, ctypes.c_int, ctypes.POINTER(_ExploreResult),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(u64)]
        L.gx_server_get_stats.restype = st
        L.gx_server_get_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
        L.gx_server_destroy.restype = st
        L.gx_server_destroy.argtypes = [vp]
        _lib_handle = L
    return _lib_handle


def status_str(code: int) -> str:
    return lib().gx_status_str(code).decode()


def _check(code: int, what: str) -> None:
    if code != GX_OK:
        raise GxError(code, what)


def _stream_handle(stream) -> int:
    import torch

    if stream is None:
        # torch's current stream, as a raw handle (without building a Stream
        # object where torch offers that)
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return int(raw(torch.cuda.current_device()) or 0)
        stream = torch.cuda.current_stream()
    return int(getattr(stream, "cuda_stream", stream) or 0)


def _dev_ptr(t, what: str) -> int:
    if t is None:
        return 0
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return int(t.data_ptr())


# ------------------------------------------------------------------ table
@dataclass
class TableInfo:
    words_per_state: int
    slot_words: int
    bucket_words: int
    subgroup: int
    keys_per_subgroup: int
    max_hashes: int
    n_buckets: int
    n_slots: int
    hash_seed: int
    bytes: int


@dataclass
class Stats:
    stored: int
    lookups: int
    probes: int
    full: int
    invalid: int
    max_hash_index: int


class Table:
    """gx_table: a bucketed find-or-put table in device memory."""

    def __init__(self, words_per_state: int, bucket_words: int, capacity: int, *,
                 hash_seed: int = 0, max_hashes: int = 0, subgroup: int = 0,
                 keys_per_subgroup: int = 0):
        opts = _TableOpts(hash_seed, max_hashes, subgroup, keys_per_subgroup, 0)
        h = ctypes.c_void_p()
        _check(lib().gx_table_create(words_per_state, bucket_words, capacity,
                                     ctypes.byref(opts), ctypes.byref(h)), "gx_table_create")
        self._destroy = lib().gx_table_destroy
        self._h = h
        self.info = self._info()

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("table destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            # the destroy function is held by the object: at interpreter exit
            # the module's globals may already be gone when __del__ runs
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _info(self) -> TableInfo:
        i = _TableInfo()
        _check(lib().gx_table_get_info(self.handle, ctypes.byref(i)), "gx_table_get_info")
        return TableInfo(i.words_per_state, i.slot_words, i.bucket_words, i.subgroup,
                         i.keys_per_subgroup, i.max_hashes, i.n_buckets, i.n_slots,
                         i.hash_seed, i.bytes)

    def clear(self, stream=None) -> None:
        _check(lib().gx_table_clear(self.handle, _stream_handle(stream)), "gx_table_clear")

    def find_or_put(self, keys, status, n_new=None, stream=None) -> None:
        """keys: device int32/uint32 tensor (n, w); status: device uint8 (n,);
        n_new: optional device int64 (1,) to which the NEW count is added."""
        n = keys.shape[0] if keys.dim() > 0 else 0
        if keys.dim() != 2 or keys.shape[1] != self.info.words_per_state:
            raise ValueError("keys must have shape (n, words_per_state)")
        if status.numel() < n:
            raise ValueError("status too small")
        _check(lib().gx_find_or_put(self.handle, _dev_ptr(keys, "keys"), n,
                                    _dev_ptr(status, "status"), _dev_ptr(n_new, "n_new"),
                                    _stream_handle(stream)), "gx_find_or_put")

    def stats(self) -> Stats:
        s = _Stats()
        _check(lib().gx_table_stats(self.handle, ctypes.byref(s)), "gx_table_stats")
        return Stats(s.stored, s.lookups, s.probes, s.full, s.invalid, s.max_hash_index)

    def dump(self) -> np.ndarray:
        """Stored keys, sorted lexicographically, shape (n, w) uint32."""
        n = ctypes.c_uint64()
        code = lib().gx_table_dump(self.handle, None, 0, ctypes.byref(n))
        if code not in (GX_OK, GX_ENOMEM):
            _check(code, "gx_table_dump")
        out = np.empty((n.value, self.info.words_per_state), dtype=np.uint32)
        _check(lib().gx_table_dump(self.handle, out.ctypes.data, n.value, ctypes.byref(n)),
               "gx_table_dump")
        return out

    def read_raw(self, first_word: int = 0, n_words: int | None = None) -> np.ndarray:
        total = self.info.n_buckets * self.info.bucket_words
        if n_words is None:
            n_words = total - first_word
        out = np.empty(n_words, dtype=np.uint32)
        _check(lib().gx_table_read_raw(self.handle, out.ctypes.data, first_word, n_words),
               "gx_table_read_raw")
        return out

    def copy_raw(self, out, first_word: int = 0, stream=None) -> None:
        """Copy raw storage words [first_word, first_word + out.numel()) into the
        device tensor ``out`` (int32 or uint32), stream-ordered."""
        _check(lib().gx_table_copy_raw(self.handle, _dev_ptr(out, "out"), first_word,
                                       out.numel(), _stream_handle(stream)),
               "gx_table_copy_raw")


def hash_bucket(key, words_per_state: int, hash_seed: int, j: int, n_buckets: int) -> int:
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1)
    out = ctypes.c_uint64()
    _check(lib().gx_hash_bucket(k.ctypes.data, words_per_state, hash_seed, j, n_buckets,
                                ctypes.byref(out)), "gx_hash_bucket")
    return int(out.value)


# ------------------------------------------------------------------ networks
class NetworkView:
    """ctypes view of a network object (n_states, initial, trans, n_labels,
    rules) as the library reads it; keeps its arrays alive.  Every call that
    takes a network also takes a view (network_view), so a caller that
    explores one network again and again marshals it once.  The view holds
    copies of the network's arrays: later changes to the network are not
    seen through it."""

    def __init__(self, net):
        P = len(net.n_states)
        self.n_procs = P
        self.arrays = []
        procs = (_Lts * P)()
        for p in range(P):
            t = np.ascontiguousarray(np.asarray(net.trans[p], dtype=np.uint32).reshape(-1, 3))
            src, lab, dst = (np.ascontiguousarray(t[:, i]) for i in range(3))
            self.arrays += [src, lab, dst]
            procs[p] = _Lts(int(net.n_states[p]), int(net.initial[p]), t.shape[0],
                            src.ctypes.data, lab.ctypes.data, dst.ctypes.data)
        rules = np.ascontiguousarray(np.asarray(net.rules, dtype=np.int32).reshape(-1, P))
        self.arrays += [rules, procs]
        self.c = _Network(P, procs, int(net.n_labels), rules.shape[0],
                          rules.ctypes.data if rules.size else None)


_NetHolder = NetworkView


def network_view(net) -> NetworkView:
    """The network's ctypes view, built once for repeated calls."""
    return net if isinstance(net, NetworkView) else NetworkView(net)


@dataclass
class Network:
    """A network of LTSs as the library describes it (Sec. 3): per process its
    state count, initial state and (src, label, dst) transitions, the label
    count and the rule matrix (label per process or -1)."""
    n_states: np.ndarray
    initial: np.ndarray
    trans: list
    n_labels: int
    rules: np.ndarray


def add_monitor(net, automaton, bad) -> tuple:
    """gx_network_add_monitor: the network with the automaton of a negated
    safety property as its last process (Sec. 3).  ``automaton`` is
    (n_states, initial, [(src, action, dst)]) with actions numbered as in
    gx_monitor (rule r, or n_rules + l for label l fired alone); ``bad``
    lists its bad states.  Returns (Network, monitor process, bad flags) for
    explore(..., monitor=(process, flags))."""
    n, init, trans = automaton
    t = np.asarray(trans, dtype=np.uint32).reshape(-1, 3)
    src, act, dst = (np.ascontiguousarray(t[:, i]) for i in range(3))
    flags = np.zeros(max(1, int(n)), dtype=np.uint8)
    flags[list(bad)] = 1
    h = network_view(net)
    mon = _Monitor(int(n), int(init), t.shape[0], src.ctypes.data, act.ctypes.data,
                   dst.ctypes.data, flags.ctypes.data)
    out = _MonitoredNetwork()
    _check(lib().gx_network_add_monitor(ctypes.byref(h.c), ctypes.byref(mon), ctypes.byref(out)),
           "gx_network_add_monitor")
    try:
        c = out.net
        P = int(c.n_procs)
        n_states, initial, tr = [], [], []
        for p in range(P):
            lt = c.procs[p]
            k = int(lt.n_trans)
            cols = [np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint32)),
                                          shape=(k,)).copy() if k else np.zeros(0, np.uint32)
                    for ptr in (lt.src, lt.label, lt.dst)]
            n_states.append(int(lt.n_states))
            initial.append(int(lt.initial))
            tr.append(np.stack(cols, axis=1).astype(np.uint32).reshape(-1, 3))
        R = int(c.n_rules)
        if R:
            rules = np.ctypeslib.as_array(ctypes.cast(c.rules, ctypes.POINTER(ctypes.c_int32)),
                                          shape=(R * P,)).copy().reshape(R, P)
        else:
            rules = np.zeros((0, P), np.int32)
        badf = np.ctypeslib.as_array(out.monitor_bad, shape=(n_states[-1],)).astype(bool)
        composed = Network(np.asarray(n_states, np.uint32), np.asarray(initial, np.uint32), tr,
                           int(c.n_labels), rules)
        return composed, int(out.monitor_proc), badf
    finally:
        lib().gx_monitored_network_free(ctypes.byref(out))


def network_words(net) -> int:
    h = network_view(net)
    w = ctypes.c_uint32()
    _check(lib().gx_network_words(ctypes.byref(h.c), ctypes.byref(w)), "gx_network_words")
    return int(w.value)


def network_pack(net, local) -> np.ndarray:
    h = network_view(net)
    P = h.n_procs
    loc = np.ascontiguousarray(local, dtype=np.uint32).reshape(-1, P)
    w = network_words(h)
    out = np.empty((loc.shape[0], w), dtype=np.uint32)
    _check(lib().gx_network_pack(ctypes.byref(h.c), loc.ctypes.data, loc.shape[0],
                                 out.ctypes.data), "gx_network_pack")
    return out


@dataclass
class ExploreResult:
    n_states: int
    n_transitions: int
    words_per_state: int
    levels: np.ndarray
    deadlocks: np.ndarray
    local_duplicates: int = 0
    violations: np.ndarray = None  # (n, w) uint32, sorted (safety monitor)
    violation_level: int | None = None
    states: np.ndarray = None  # (n_states, w) uint32, sorted (keep_states of batches, servers)


def _copy_out(addr, n: int, dtype) -> np.ndarray:
    """A numpy copy of n elements at a library-owned host address."""
    if not n or not addr:
        return np.zeros(0, dtype)
    return np.frombuffer(ctypes.string_at(addr, n * np.dtype(dtype).itemsize), dtype=dtype).copy()


def _take_result(res: _ExploreResult) -> ExploreResult:
    w = res.words_per_state
    levels = _copy_out(res.level_counts, res.n_levels, np.uint64)
    dead = _copy_out(res.deadlocks, res.n_deadlocks * w, np.uint32)
    viol = _copy_out(res.violations, res.n_violations * w, np.uint32)
    vl = None if res.violation_level == 0xFFFFFFFF else int(res.violation_level)
    states = None
    if res.states:
        states = _copy_out(res.states, res.n_states * w, np.uint32).reshape(-1, w)
    out = ExploreResult(int(res.n_states), int(res.n_transitions), w, levels,
                        dead.reshape(-1, w), int(res.local_duplicates), viol.reshape(-1, w), vl,
                        states)
    lib().gx_explore_result_free(ctypes.byref(res))
    return out


def explore(net, table: Table, *, frontier_capacity: int = 0, deadlock_capacity: int = 0,
            stream=None, local_dedup: bool = False, monitor=None,
            stop_on_violation: bool = False, slice_states: int = 0) -> ExploreResult:
    """gx_explore: BFS of the synchronous product into ``table``.  monitor =
    (process, bad flags per local state of it) checks a safety property;
    slice_states: most frontier states per slice of a level (0: 2^22)."""
    h = network_view(net)
    proc, bad = 0, None
    if monitor is not None:
        proc = int(monitor[0])
        bad = np.ascontiguousarray(np.asarray(monitor[1]).astype(np.uint8))
        if not 0 <= proc < h.n_procs or bad.shape != (int(h.c.procs[proc].n_states),):
            raise ValueError("monitor: a process index and one flag per local state of it")
    opts = _ExploreOpts(frontier_capacity, deadlock_capacity, _stream_handle(stream),
                        int(local_dedup), proc, int(stop_on_violation), int(slice_states),
                        bad.ctypes.data if bad is not None else None)
    res = _ExploreResult()
    _check(lib().gx_explore(ctypes.byref(h.c), table.handle, ctypes.byref(opts),
                            ctypes.byref(res)), "gx_explore")
    return _take_result(res)


def explore_noalloc(net, table: Table, *, max_levels: int = 4096, max_deadlocks: int = 1 << 20,
                    frontier_capacity: int = 0, deadlock_capacity: int = 0, stream=None,
                    local_dedup: bool = False) -> ExploreResult:
    """gx_explore_noalloc: gx_explore with the library's static scratch array
    for its device buffers and results in host arrays passed in (here numpy
    arrays of max_levels and max_deadlocks entries)."""
    h = network_view(net)
    w = table.info.words_per_state
    levels = np.zeros(max(1, max_levels), dtype=np.uint64)
    dead = np.zeros((max(1, max_deadlocks), w), dtype=np.uint32)
    opts = _ExploreOpts(frontier_capacity, deadlock_capacity, _stream_handle(stream),
                        int(local_dedup), 0, 0, 0, None)
    summ = _ExploreSummary()
    _check(lib().gx_explore_noalloc(ctypes.byref(h.c), table.handle, ctypes.byref(opts),
                                    levels.ctypes.data, max_levels, dead.ctypes.data,
                                    max_deadlocks, ctypes.byref(summ)), "gx_explore_noalloc")
    return ExploreResult(int(summ.n_states), int(summ.n_transitions), w,
                         levels[: summ.n_levels].copy(), dead[: summ.n_deadlocks].copy())


def gather_probe(buf, granule: int, n_reads: int, seed: int, sink, stream=None) -> None:
    """gx_gather_probe over a device tensor ``buf``; ``sink``: device int64 (1,)."""
    _check(lib().gx_gather_probe(_dev_ptr(buf, "buf"), buf.numel() * buf.element_size(),
                                 granule, n_reads, seed, _dev_ptr(sink, "sink"),
                                 _stream_handle(stream)), "gx_gather_probe")


def claim_probe(buf, mode: int, n_ops: int, seed: int, sink, stream=None) -> None:
    """gx_claim_probe on a device tensor `buf` (1: compare-and-swaps, 2: reads
    with a compare-and-swap for every other one); sink: a device int64 tensor."""
    _check(lib().gx_claim_probe(buf.data_ptr(), buf.numel() * buf.element_size(), mode, n_ops,
                                seed, sink.data_ptr(), _stream_handle(stream)), "gx_claim_probe")


# ------------------------------------------------------------------ batches
def autotune(words_per_state: int, load_factor: float = 0.5) -> tuple[int, int, int]:
    """gx_autotune: (bucket_words, subgroup, keys_per_subgroup) measured best."""
    b, g, u = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().gx_autotune(words_per_state, load_factor, ctypes.byref(b), ctypes.byref(g),
                             ctypes.byref(u)), "gx_autotune")
    return int(b.value), int(g.value), int(u.value)


def autotune_capacity(words_per_state: int, capacity: int, load_factor: float = 0.5) -> dict:
    """gx_autotune_capacity: the pick for tables of `capacity` states, with the
    timings behind it (ns per key of the pick, the default and the runner-up)."""
    t = _TuneInfo()
    _check(lib().gx_autotune_capacity(words_per_state, load_factor, capacity, ctypes.byref(t)),
           "gx_autotune_capacity")
    return {n: getattr(t, n) for n, _ in _TuneInfo._fields_ if n != "pad"}


class Batch:
    """gx_batch: many explorations together, level-synchronous steps over all
    unfinished instances (the default), or one persistent launch per kernel
    class pulling work from a device queue (``persistent`` or ``use_graph``)."""

    def __init__(self, nets, capacity, *, hash_seed: int = 0, max_hashes: int = 0,
                 bucket_words: int = 0, subgroup: int = 0, keys_per_subgroup: int = 0,
                 use_graph: bool = False, max_levels: int = 0, deadlock_capacity: int = 0,
                 keep_states: bool = False, persistent: bool = False):
        self.n = len(nets)
        holders = [network_view(net) for net in nets]
        arr = (_Network * self.n)(*[h.c for h in holders])
        cap = np.ascontiguousarray(capacity, dtype=np.uint64).reshape(-1)
        if cap.shape[0] != self.n:
            raise ValueError("one capacity per network")
        opts = _BatchOpts(cap.ctypes.data, hash_seed, max_hashes, bucket_words, subgroup,
                          keys_per_subgroup, int(use_graph), max_levels, deadlock_capacity, None,
                          int(keep_states), int(persistent))
        h = ctypes.c_void_p()
        _check(lib().gx_batch_create(arr, self.n, ctypes.byref(opts), ctypes.byref(h)),
               "gx_batch_create")
        self._destroy = lib().gx_batch_destroy
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            # the destroy function is held by the object: at interpreter exit
            # the module's globals may already be gone when __del__ runs
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, stream=None) -> None:
        _check(lib().gx_batch_run(self._h, _stream_handle(stream)), "gx_batch_run")

    def results(self):
        """List of (status, ExploreResult or None), one per instance."""
        outs = (_ExploreResult * self.n)()
        sts = (ctypes.c_int * self.n)()
        _check(lib().gx_batch_results(self._h, outs, sts), "gx_batch_results")
        return [(int(sts[i]), _take_result(outs[i]) if sts[i] == GX_OK else None)
                for i in range(self.n)]

    def instance_config(self, i: int) -> tuple[int, int, int]:
        b, g, u = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().gx_batch_instance_config(self._h, i, ctypes.byref(b), ctypes.byref(g),
                                              ctypes.byref(u)), "gx_batch_instance_config")
        return int(b.value), int(g.value), int(u.value)


def explore_batch(nets, capacity, stream=None, **opts):
    """gx_explore_batch: create, run, collect and destroy in one call."""
    with Batch(nets, capacity, **opts) as b:
        b.run(stream)
        return b.results()


# ------------------------------------------------------------------ serving
class Server:
    """gx_server: admission by HBM reservation, resident tables, continuous
    batching of exploration requests at BFS-level granularity."""

    def __init__(self, budget_bytes: int, *, max_active: int = 0, max_hashes: int = 0,
                 load_factor: float = 0.0, hash_seed: int = 0, bucket_words: int = 0,
                 subgroup: int = 0, keys_per_subgroup: int = 0, keep_states: bool = False):
        opts = _ServerOpts(budget_bytes, max_active, max_hashes, load_factor, hash_seed,
                           bucket_words, subgroup, keys_per_subgroup, int(keep_states))
        h = ctypes.c_void_p()
        _check(lib().gx_server_create(ctypes.byref(opts), ctypes.byref(h)), "gx_server_create")
        self._destroy = lib().gx_server_destroy
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            # the destroy function is held by the object: at interpreter exit
            # the module's globals may already be gone when __del__ runs
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, net, declared_states: int) -> int:
        h = network_view(net)
        rid = ctypes.c_uint64()
        _check(lib().gx_server_submit(self._h, ctypes.byref(h.c), declared_states,
                                      ctypes.byref(rid)), "gx_server_submit")
        return int(rid.value)

    def poll(self, request_id: int, wait: bool = True):
        """(status, ExploreResult or None, latency in seconds), or None while
        the request runs (wait=False)."""
        res = _ExploreResult()
        st = ctypes.c_int()
        lat = ctypes.c_uint64()
        code = lib().gx_server_poll(self._h, request_id, int(wait), ctypes.byref(res),
                                    ctypes.byref(st), ctypes.byref(lat))
        if code == GX_EBUSY:
            return None
        _check(code, "gx_server_poll")
        out = _take_result(res) if st.value == GX_OK else None
        return int(st.value), out, lat.value * 1e-9

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().gx_server_get_stats(self._h, ctypes.byref(s)), "gx_server_get_stats")
        return {n: int(getattr(s, n)) for n, _ in _ServerStats._fields_}
