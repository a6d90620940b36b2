"""CPU-only checks of the C-ABI library: it loads, exports every declared
entry point, rejects invalid arguments before touching a device, and its host
logic (packing plan, hash family) matches independent implementations."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gx_status|void|const char\s*\*)\s*(gx_\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gx.LIB_PATH):
        from paper_1801_05857_amd import build

        build.build(force=False)
    return gx.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gx.EXPORTED)


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert gx.status_str(code).startswith("GX_")


@pytest.mark.parametrize("w,B,cap,sub,kps", [
    (0, 32, 10, 0, 0), (5, 32, 10, 0, 0), (1, 12, 10, 0, 0), (1, 2, 10, 0, 0),
    (1, 128, 10, 0, 0), (2, 32, 0, 0, 0), (2, 32, 10, 12, 0), (2, 64, 10, 4, 0), (2, 32, 10, 2, 0), (2, 32, 10, 4, 8),
    (2, 32, 10, 128, 0), (2, 32, 10, 0, 3), (2, 32, 10, 0, 16)])
def test_table_create_rejects_bad_arguments(lib, w, B, cap, sub, kps):
    opts = gx._TableOpts(0, 0, sub, kps, 0)
    h = ctypes.c_void_p()
    assert lib.gx_table_create(w, B, cap, ctypes.byref(opts), ctypes.byref(h)) == gx.GX_EINVAL
    assert not h.value  # out-parameter untouched


def test_null_handles_rejected(lib):
    assert lib.gx_find_or_put(None, None, 1, None, None, None) == gx.GX_EINVAL
    assert lib.gx_table_clear(None, None) == gx.GX_EINVAL
    assert lib.gx_table_get_info(None, None) == gx.GX_EINVAL
    assert lib.gx_table_stats(None, None) == gx.GX_EINVAL
    assert lib.gx_table_dump(None, None, 0, None) == gx.GX_EINVAL
    assert lib.gx_explore(None, None, None, None) == gx.GX_EINVAL
    assert lib.gx_table_destroy(None) == gx.GX_OK
    assert lib.gx_gather_probe(None, 0, 64, 1, 0, None, None) == gx.GX_EINVAL
    assert lib.gx_claim_probe(None, 64, 1, 1, 0, None, None) == gx.GX_EINVAL
    buf = ctypes.c_void_p(64)
    assert lib.gx_claim_probe(buf, 32, 1, 1, 0, buf, None) == gx.GX_EINVAL   # too small
    assert lib.gx_claim_probe(buf, 4096, 3, 1, 0, buf, None) == gx.GX_EINVAL  # no mode 3
    assert lib.gx_claim_probe(ctypes.c_void_p(72), 4096, 1, 1, 0, buf, None) == gx.GX_EINVAL


def _bad_nets():
    good = W.fig1_producer_consumers()
    yield "label out of range", W.Network(good.n_states, good.initial,
                                          [np.array([[0, 9, 1]], np.uint32)] + good.trans[1:],
                                          good.n_labels, good.rules)
    yield "target out of range", W.Network(good.n_states, good.initial,
                                           [np.array([[0, 1, 2]], np.uint32)] + good.trans[1:],
                                           good.n_labels, good.rules)
    yield "initial out of range", W.Network(good.n_states, np.array([2, 0, 0], np.uint32),
                                            good.trans, good.n_labels, good.rules)
    yield "empty rule", W.Network(good.n_states, good.initial, good.trans, good.n_labels,
                                  np.array([[-1, -1, -1]], np.int32))
    yield "rule label out of range", W.Network(good.n_states, good.initial, good.trans,
                                               good.n_labels, np.array([[7, -1, -1]], np.int32))
    big = 2**30 + 1  # 31-bit fields: five of them need five words
    yield "five words", W.Network(np.full(5, big, np.uint32), np.zeros(5, np.uint32),
                                  [np.zeros((0, 3), np.uint32)] * 5, 1,
                                  np.zeros((0, 5), np.int32))


@pytest.mark.parametrize("what,net", list(_bad_nets()))
def test_invalid_networks(lib, what, net):
    with pytest.raises(gx.GxError) as e:
        gx.network_words(net)
    assert e.value.code == gx.GX_EINVAL


@pytest.mark.parametrize("seed", range(12))
def test_packing_matches_oracle(lib, seed):
    rng = W.SplitMix64(seed)
    P = 1 + rng.below(14)
    ns = [1 + rng.below(300) for _ in range(P)]
    net = W.random_lts(seed, P, ns, ns, out_degree=1, n_labels=4)
    assert gx.network_words(net) == oracle.pack_plan(ns)[0]
    local = np.array([[rng.below(n) for n in ns] for _ in range(20)], dtype=np.uint32)
    assert np.array_equal(gx.network_pack(net, local), oracle.pack(ns, local))


def test_packing_golden_token_ring(lib):
    # Sec. 5.2: 10 nodes fit one word, 11 need two
    assert gx.network_words(W.token_ring(10)) == 1
    assert gx.network_words(W.token_ring(11)) == 2
    assert gx.network_words(W.random_lts(1, 12, 64, 8)) == 3


# ---------------------------------------------------------------- hash family
M64 = (1 << 64) - 1
DEFAULT_SEED = 0x1801058570


def _fmix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _bucket(key, w, seed, j, nb):
    # h_j(k) = mulhi64(a_j * m(k) + c_j, n_buckets), from the documented family
    seed = seed or DEFAULT_SEED
    k = list(key) + [0] * (4 - len(key))
    x = k[0] | ((k[1] << 32) if w >= 2 else 0)
    if w >= 3:
        x = _fmix(x ^ seed) ^ (k[2] | (k[3] << 32))
    m = _fmix(x ^ seed)
    a = _fmix((seed + (2 * j + 1) * 0x9E3779B97F4A7C15) & M64) | 1
    c = _fmix((seed + (2 * j + 2) * 0x9E3779B97F4A7C15) & M64)
    return (((a * m + c) & M64) * nb) >> 64


@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_hash_family_matches_definition(lib, w):
    rng = np.random.default_rng(w)
    for _ in range(200):
        key = rng.integers(0, 2**31, size=w).tolist()
        seed = int(rng.integers(0, 2**63))
        j = int(rng.integers(0, 16))
        nb = int(rng.integers(1, 2**40))
        assert gx.hash_bucket(key, w, seed, j, nb) == _bucket(key, w, seed, j, nb)


def test_hash_family_spreads_keys(lib):
    # 64k sequential keys over 1024 buckets: every bucket used, max load small
    nb = 1024
    loads = np.zeros(nb, np.int64)
    for i in range(1 << 16):
        loads[gx.hash_bucket([i, 0], 2, 0, 0, nb)] += 1
    assert loads.min() > 0 and loads.max() < 4 * (1 << 16) // nb


def test_batch_arguments_rejected_before_device_work(lib):
    net = W.fig1_producer_consumers()
    h = gx._NetHolder(net)
    arr = (gx._Network * 1)(h.c)
    cap = np.array([0], np.uint64)
    opts = gx._BatchOpts(cap.ctypes.data, 0, 0, 0, 0, 0, 0, 0, 0, None)
    out = ctypes.c_void_p()
    assert lib.gx_batch_create(arr, 1, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    cap[0] = 10
    opts = gx._BatchOpts(cap.ctypes.data, 0, 0, 12, 0, 0, 0, 0, 0, None)
    assert lib.gx_batch_create(arr, 1, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._BatchOpts(cap.ctypes.data, 0, 0, 0, 32, 0, 0, 0, 0, None)
    assert lib.gx_batch_create(arr, 1, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    # a 4-lane subgroup covers at most 32 bucket words
    opts = gx._BatchOpts(cap.ctypes.data, 0, 0, 64, 4, 0, 0, 0, 0, None)
    assert lib.gx_batch_create(arr, 1, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._BatchOpts(cap.ctypes.data, 0, 0, 0, 2, 0, 0, 0, 0, None)
    assert lib.gx_batch_create(arr, 1, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    assert lib.gx_batch_create(arr, 0, ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    assert not out.value
    assert lib.gx_batch_run(None, None) == gx.GX_EINVAL
    assert lib.gx_batch_results(None, None, None) == gx.GX_EINVAL
    b = ctypes.c_uint32()
    assert lib.gx_autotune(0, 0.5, ctypes.byref(b), ctypes.byref(b), ctypes.byref(b)) == gx.GX_EINVAL
    assert lib.gx_autotune(2, 0.0, ctypes.byref(b), ctypes.byref(b), ctypes.byref(b)) == gx.GX_EINVAL
    t = gx._TuneInfo()
    assert lib.gx_autotune_capacity(0, 0.5, 1024, ctypes.byref(t)) == gx.GX_EINVAL
    assert lib.gx_autotune_capacity(2, 0.96, 1024, ctypes.byref(t)) == gx.GX_EINVAL
    assert lib.gx_autotune_capacity(2, 0.5, 0, ctypes.byref(t)) == gx.GX_EINVAL
    assert lib.gx_autotune_capacity(2, 0.5, 1024, None) == gx.GX_EINVAL


def test_server_arguments_rejected(lib):
    out = ctypes.c_void_p()
    assert lib.gx_server_create(None, ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._ServerOpts(0, 0, 0, 0.0, 0, 0, 0, 0, 0)
    assert lib.gx_server_create(ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._ServerOpts(1 << 20, 0, 0, 0.99, 0, 0, 0, 0, 0)
    assert lib.gx_server_create(ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._ServerOpts(1 << 20, 0, 0, 0.5, 0, 12, 0, 0, 0)
    assert lib.gx_server_create(ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._ServerOpts(1 << 20, 0, 0, 0.5, 0, 64, 4, 0, 0)
    assert lib.gx_server_create(ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    opts = gx._ServerOpts(1 << 20, 0, 0, 0.5, 0, 0, 32, 0, 0)
    assert lib.gx_server_create(ctypes.byref(opts), ctypes.byref(out)) == gx.GX_EINVAL
    assert not out.value
    rid = ctypes.c_uint64()
    assert lib.gx_server_submit(None, None, 10, ctypes.byref(rid)) == gx.GX_EINVAL
    assert lib.gx_server_destroy(None) == gx.GX_OK


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with status 2 and
    a JSON error line, before any device is touched."""
    import json
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "--gpus must be 1" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def test_networks_with_images_beyond_lds_compile(lib):
    """A network whose compiled image exceeds the 46 KiB LDS budget still
    compiles for gx_explore (its image is then read from global memory):
    its words and packing are available on the host."""
    import workloads as W
    net = W.random_lts(21, 4, 4096, 12, 3, 32, 0.25, 0.1)  # 4 x 4097 offsets alone
    assert gx.network_words(net) == 2
    packed = gx.network_pack(net, np.zeros((1, 4), dtype=np.uint32))
    assert packed.shape == (1, 2) and not packed.any()


def test_network_view_is_accepted_wherever_a_network_is(lib):
    """network_view builds the ctypes view once; the host-side calls take it
    in place of the network."""
    net = W.random_lts(21, 4, 4096, 12, 3, 32, 0.25, 0.1)
    v = gx.network_view(net)
    assert gx.network_view(v) is v
    assert gx.network_words(v) == gx.network_words(net) == 2
    loc = np.array([[1, 2, 3, 4]], dtype=np.uint32)
    assert np.array_equal(gx.network_pack(v, loc), gx.network_pack(net, loc))
