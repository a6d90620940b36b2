"""Parity of gx_explore on the large plain-path workload: 12 processes of 64
declared states (3-word vectors), 3.3e9 reachable states in a 192 GB table,
explored in the configuration the benchmark times (buckets of 32 words,
subgroups of 8 lanes, one key in flight per subgroup).

The oracle cannot enumerate 3.3e9 states, so at full size the result is
checked by what the oracle can compute exactly and by properties that hold at
any size:
* the first BFS levels (a prefix of up to ~300 thousand states) equal the
  oracle's level counts on the same network;
* level counts add up to the state count, which equals the number of keys
  the table stored, with no table overflow;
* closure on samples: for states sampled from the final table, every
  successor the oracle computes is already stored (a find-or-put of all of
  them returns SEEN and stores nothing);
* every sampled stored state decodes to local states within their processes;
* deadlocks: the network has none, and the oracle finds none among the
  sampled states.
The same network family at a size the oracle enumerates (4 live states per
process) is compared bit-exactly, table contents included."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

STATES_FULL = 3_304_390_656


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def test_same_family_at_oracle_size_bit_exact(dev):
    net = W.large_random_network(live=4)
    want = oracle.explore(net, want_visited=True)
    with gx.Table(3, 32, 2 * want.n_states, subgroup=8, keys_per_subgroup=1,
                  max_hashes=16) as t:
        got = gx.explore(net, t)
        assert got.n_states == want.n_states == 248832
        assert got.levels.tolist() == want.levels.tolist()
        assert got.n_transitions == want.n_transitions
        assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)


def _sample_stored(t, rng, n_windows=64, window_words=1 << 14, want=4096):
    """States read from random windows of the raw table (slot format, S = 4)."""
    info = t.info
    total = info.n_buckets * info.bucket_words
    out = []
    for _ in range(n_windows):
        first = int(rng.integers(0, total - window_words)) // 4 * 4
        raw = t.read_raw(first, window_words).reshape(-1, 4)
        occ = raw[raw[:, 0] != 0xFFFFFFFF]
        out.append(occ[:, :3])
    s = np.concatenate(out)
    return s[: want]


def test_full_size_properties(dev):
    torch.cuda.empty_cache()  # room for the 192 GB table
    net = W.large_random_network()
    with gx.Table(3, 32, W.LARGE_TABLE_SLOTS, subgroup=8, keys_per_subgroup=1,
                  max_hashes=16) as t:
        r = gx.explore(net, t)
        assert r.n_states == STATES_FULL
        lv = r.levels
        assert lv[0] == 1 and (lv > 0).all() and int(lv.sum()) == r.n_states
        s = t.stats()
        assert s.stored == r.n_states and s.full == 0
        assert len(r.deadlocks) == 0

        # BFS prefix against the oracle
        k = int(np.searchsorted(np.cumsum(lv), 300_000, side="right"))
        assert k >= 5
        pre = oracle.explore(net, max_levels=k)
        assert pre.levels.tolist() == lv[:k].tolist()

        # closure on samples
        rng = np.random.default_rng(1801058570)
        sample = _sample_stored(t, rng)
        assert sample.shape[0] >= 1024
        counts, succ = oracle.successors(net, sample)  # raises on an invalid state
        assert (counts > 0).all()  # no deadlock among them
        keys = torch.from_numpy(np.ascontiguousarray(succ).view(np.int32)).to(dev)
        st = torch.full((keys.shape[0],), 255, dtype=torch.uint8, device=dev)
        n_new = torch.zeros(1, dtype=torch.int64, device=dev)
        t.find_or_put(keys, st, n_new)
        torch.cuda.synchronize()
        assert int(n_new.item()) == 0
        assert bool((st == gx.GX_SEEN).all().item())
