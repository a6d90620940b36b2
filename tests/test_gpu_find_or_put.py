"""GPU parity of gx_find_or_put against the oracle (set insertion).

Several results are correct when a key occurs more than once among keys that
were absent before a call (which occurrence is reported NEW is unspecified), so
the comparison is on what is unique: the exact NEW count, exactly one NEW per
absent distinct key, SEEN for every key present before the call, and the final
table contents as a set.  Placement is checked against the hash sequence.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

from setdigest import P, digest_words, table_digest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def _run(table, keys_np, dev):
    k = torch.from_numpy(np.ascontiguousarray(keys_np).view(np.int32)).to(dev)
    st = torch.full((max(1, k.shape[0]),), 255, dtype=torch.uint8, device=dev)
    n_new = torch.zeros(1, dtype=torch.int64, device=dev)
    table.find_or_put(k, st[: k.shape[0]], n_new)
    torch.cuda.synchronize()
    return st[: k.shape[0]].cpu().numpy(), int(n_new.item())


def _check_batch(keys, status, present_before):
    """Per distinct key: SEEN everywhere if it was present before, else exactly
    one NEW among its occurrences."""
    assert set(np.unique(status).tolist()) <= {gx.GX_NEW, gx.GX_SEEN}
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    new_per_key = np.bincount(inv, weights=(status == gx.GX_NEW), minlength=uniq.shape[0])
    was = np.array([present_before(u) for u in uniq], dtype=bool)
    assert (new_per_key[was] == 0).all()
    assert (new_per_key[~was] == 1).all()
    return int((~was).sum())


def _placement_ok(table, keys_sorted):
    """Every stored key sits in bucket h_j(key) for some j, with the buckets of
    h_0 .. h_{j-1} full and every lower slot of its own bucket occupied."""
    info = table.info
    raw = table.read_raw().reshape(info.n_buckets, info.bucket_words)
    S, w, B = info.slot_words, info.words_per_state, info.bucket_words
    slots = raw.reshape(info.n_buckets, B // S, S)
    occupied = slots[:, :, 0] != gx.EMPTY_WORD
    full = occupied.all(axis=1)
    where = {}
    for b, s in zip(*np.nonzero(occupied)):
        where[tuple(slots[b, s, :w].tolist())] = (b, s)
    assert len(where) == keys_sorted.shape[0]
    for key in keys_sorted:
        b, s = where[tuple(key.tolist())]
        assert occupied[b, :s].all()
        for j in range(info.max_hashes):
            hb = gx.hash_bucket(key, w, info.hash_seed, j, info.n_buckets)
            if hb == b:
                break
            assert full[hb], "an earlier bucket of the hash sequence had room"
        else:
            raise AssertionError("key stored outside its hash sequence")
        if S == 4 and w == 3:
            assert slots[b, s, 3] == 0


GRID = [(w, B, G, U) for w in (1, 2, 3, 4) for B in (4, 8, 16, 32, 64) for G in (8, 16, 32, 64)
        for U in (1, 2, 4, 8)]
# 4-lane subgroups: buckets of at most 32 words (8 per lane), U <= 4
GRID += [(w, B, 4, U) for w in (1, 2, 3, 4) for B in (4, 8, 16, 32) for U in (1, 2, 4)]


@pytest.mark.parametrize("w,B,G,U", GRID, ids=[f"w{w}-B{B}-G{G}-U{U}" for w, B, G, U in GRID])
def test_specialisation_parity(dev, w, B, G, U):
    n_distinct = 3000
    keys = W.duplicated_stream(n_distinct, 3, w, seed=w * 1000 + B + G + U)
    ref = oracle.OracleSet(w)
    # both batches together hold about 2.5 * n_distinct keys: load factor < 0.2
    with gx.Table(w, B, 16 * n_distinct, subgroup=G, keys_per_subgroup=U,
                  max_hashes=32) as t:
        st, n_new = _run(t, keys, dev)
        fresh = _check_batch(keys, st, lambda k: False)
        _, ref_new = ref.insert(keys)
        assert n_new == ref_new == fresh == n_distinct
        # second batch: half old keys, half new ones, shuffled together
        more = W.distinct_keys(2 * n_distinct, w, seed=777 + w)[n_distinct // 2:]
        batch2 = np.concatenate([keys[: n_distinct], more, more[:100]])
        before = ref.dump()
        before_set = {tuple(r) for r in before.tolist()}
        st2, n_new2 = _run(t, batch2, dev)
        fresh2 = _check_batch(batch2, st2, lambda k: tuple(k.tolist()) in before_set)
        _, ref_new2 = ref.insert(batch2)
        assert n_new2 == ref_new2 == fresh2
        dump = t.dump()
        assert np.array_equal(dump, ref.dump())
        s = t.stats()
        assert s.stored == len(ref) and s.full == 0 and s.invalid == 0
        assert s.lookups == keys.shape[0] + batch2.shape[0]
        if (G, U) in ((8, 1), (64, 4), (4, 1)):
            _placement_ok(t, dump)


def test_empty_batch(dev):
    with gx.Table(2, 32, 100) as t:
        k = torch.zeros((0, 2), dtype=torch.int32, device=dev)
        st = torch.zeros(0, dtype=torch.uint8, device=dev)
        t.find_or_put(k, st)
        torch.cuda.synchronize()
        assert t.stats().lookups == 0 and t.dump().shape == (0, 2)


@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_invalid_words_rejected_per_key(dev, w):
    keys = W.distinct_keys(64, w, seed=5)
    keys[::7, w - 1] = gx.EMPTY_WORD
    with gx.Table(w, 16, 256) as t:
        st, n_new = _run(t, keys, dev)
        bad = (keys == gx.EMPTY_WORD).any(axis=1)
        assert (st[bad] == gx.GX_INVALID).all()
        assert (st[~bad] == gx.GX_NEW).all()
        assert n_new == int((~bad).sum())
        assert t.stats().invalid == int(bad.sum())
        assert t.dump().shape[0] == int((~bad).sum())


@pytest.mark.parametrize("S_w,B", [(1, 8), (2, 16), (4, 32)])
def test_full_when_hash_sequence_exhausted(dev, S_w, B):
    # one bucket, one hash function: the first B/S distinct keys fit, the rest are FULL
    w = S_w
    slots = B // (4 if w >= 3 else w)
    keys = W.distinct_keys(5 * slots, w, seed=9)
    with gx.Table(w, B, 1, max_hashes=1) as t:
        assert t.info.n_buckets == 1
        st, n_new = _run(t, keys, dev)
        assert n_new == slots
        assert int((st == gx.GX_NEW).sum()) == slots
        assert int((st == gx.GX_FULL).sum()) == 4 * slots
        s = t.stats()
        assert s.full == 4 * slots and s.stored == slots
        stored = t.dump()
        assert stored.shape[0] == slots
        # the stored keys are among the inserted ones, each once
        assert np.unique(stored, axis=0).shape[0] == slots
        # re-inserting a stored key is SEEN, a FULL one stays FULL
        st2, _ = _run(t, np.concatenate([stored[:1], keys[st == gx.GX_FULL][:1]]), dev)
        assert st2.tolist() == [gx.GX_SEEN, gx.GX_FULL]


@pytest.mark.parametrize("w,G", [(1, 8), (2, 16), (3, 8), (4, 64)])
def test_every_lane_inserts_one_key(dev, w, G):
    keys = np.repeat(W.distinct_keys(1, w, seed=3), 200_000, axis=0)
    with gx.Table(w, 32, 1024, subgroup=G, keys_per_subgroup=4) as t:
        st, n_new = _run(t, keys, dev)
        assert n_new == 1 and int((st == gx.GX_NEW).sum()) == 1
        assert int((st == gx.GX_SEEN).sum()) == keys.shape[0] - 1
        assert np.array_equal(t.dump(), keys[:1])


def _colliding_keys(w, n_buckets, want, seed):
    """Distinct keys whose first hash is bucket 0 (searched on the host)."""
    out = []
    cand = W.distinct_keys(want * n_buckets * 4, w, seed=seed)
    for k in cand:
        if gx.hash_bucket(k, w, 0, 0, n_buckets) == 0:
            out.append(k)
            if len(out) == want:
                break
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("w,B,G", [(1, 8, 8), (2, 8, 8), (2, 64, 16), (4, 16, 8), (3, 32, 32)])
def test_contended_bucket_overflows_in_order(dev, w, B, G):
    # many distinct keys, all hashing first to bucket 0, each inserted 50 times
    nb = 64
    slots_per_bucket = B // (4 if w >= 3 else w)
    base = _colliding_keys(w, nb, 3 * slots_per_bucket, seed=21 + w)
    keys = np.repeat(base, 50, axis=0)
    keys = keys[W.permutation(keys.shape[0], 5).astype(np.int64)]
    with gx.Table(w, B, nb * slots_per_bucket, subgroup=G, max_hashes=16) as t:
        assert t.info.n_buckets == nb
        st, n_new = _run(t, keys, dev)
        _check_batch(keys, st, lambda k: False)
        assert n_new == base.shape[0]
        dump = t.dump()
        assert np.array_equal(dump, np.unique(base, axis=0))
        _placement_ok(t, dump)


@pytest.mark.parametrize("B,G", [(8, 8), (16, 16), (64, 8), (64, 64)])
def test_four_word_keys_sharing_heads(dev, B, G):
    # keys that agree on words 0-1 and differ in words 2-3: the head CAS is
    # contended by different keys and the tails decide
    n = 40
    heads = W.distinct_keys(3, 2, seed=1)
    tails = W.distinct_keys(n, 2, seed=2)
    base = np.concatenate([np.repeat(heads, n, axis=0), np.tile(tails, (3, 1))], axis=1)
    keys = np.repeat(base, 30, axis=0)
    keys = keys[W.permutation(keys.shape[0], 8).astype(np.int64)]
    with gx.Table(4, B, 4 * base.shape[0], subgroup=G, max_hashes=32) as t:
        st, n_new = _run(t, keys, dev)
        _check_batch(keys, st, lambda k: False)
        assert n_new == base.shape[0]
        assert np.array_equal(t.dump(), np.unique(base, axis=0))


def test_clear_resets(dev):
    keys = W.distinct_keys(1000, 2, seed=4)
    with gx.Table(2, 16, 4000) as t:
        _run(t, keys, dev)
        t.clear()
        torch.cuda.synchronize()
        assert t.stats().stored == 0 and t.dump().shape[0] == 0
        st, n_new = _run(t, keys, dev)
        assert n_new == 1000 and (st == gx.GX_NEW).all()


def test_load_factor_09_needs_long_sequences(dev):
    # alpha = 0.9 with 4 slots per bucket: H = 8 leaves FULL keys, H = 128 does not
    n = 1 << 18
    keys = W.distinct_keys(n, 2, seed=13)
    cap = int(np.ceil(n / 0.9))
    with gx.Table(2, 8, cap, max_hashes=128) as t:
        st, n_new = _run(t, keys, dev)
        assert n_new == n and (st == gx.GX_NEW).all()
        s = t.stats()
        assert s.full == 0 and s.max_hash_index > 8
        assert t.dump().shape[0] == n


@pytest.mark.parametrize("B,G,U", [(32, 4, 1), (16, 4, 1), (16, 16, 4)])
def test_full_size_microbenchmark_properties(dev, B, G, U):
    """The 2^28-key, 2^27-distinct stream at load factor 0.5, first in the
    launch configuration the benchmark times (buckets of 32 words, 4-lane
    subgroups, one key in flight): exact NEW count, exactly one NEW per
    distinct key, the table holds exactly the distinct keys (count and set
    digest: the stream holds every distinct key twice, so its digest is twice
    the set's), every key findable afterwards, and fresh keys still NEW."""
    n_distinct = 1 << 27
    keys, idx = W.duplicated_stream_torch(n_distinct, 2, 1801058570, dev)
    with gx.Table(2, B, 2 * n_distinct, subgroup=G, keys_per_subgroup=U) as t:
        st = torch.empty(keys.shape[0], dtype=torch.uint8, device=dev)
        n_new = torch.zeros(1, dtype=torch.int64, device=dev)
        t.find_or_put(keys, st, n_new)
        torch.cuda.synchronize()
        assert int(n_new.item()) == n_distinct
        assert int((st == gx.GX_NEW).sum().item()) == n_distinct
        per_key = torch.bincount(idx[st == gx.GX_NEW], minlength=n_distinct)
        assert int(per_key.min().item()) == 1 and int(per_key.max().item()) == 1
        del per_key
        s = t.stats()
        assert s.stored == n_distinct and s.full == 0
        n_tab, d_tab = table_digest(t, dev)
        d_stream = digest_words(keys.to(torch.int64) & 0xFFFFFFFF, 2)
        assert n_tab == n_distinct
        assert d_stream == ((2 * d_tab[0]) % P, (2 * d_tab[1]) % P)
        # a sample of stored keys is found; a sample of fresh keys is new
        sample = keys[:: 1 << 8].contiguous()
        st2 = torch.empty(sample.shape[0], dtype=torch.uint8, device=dev)
        t.find_or_put(sample, st2)
        torch.cuda.synchronize()
        assert bool((st2 == gx.GX_SEEN).all().item())
        # counters seed + 2^27 .. : outside the stream's counter range, so distinct
        fresh_np = W.distinct_keys(1 << 16, 2, seed=1801058570 + (1 << 27))
        st3, _ = _run(t, fresh_np, dev)
        assert (st3 == gx.GX_NEW).all()
