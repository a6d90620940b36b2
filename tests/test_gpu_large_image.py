"""GPU parity of gx_explore on networks whose compiled image (transition
tables of every process and rule, Sec. 3) exceeds the LDS budget of the
generation kernel: the image is then read from global memory.  Bit-exact
against the oracle BFS: level counts, transitions, deadlocks and the table's
contents.  Batches and the server keep every image in LDS and refuse such
networks with GX_EINVAL; so does gx_explore_noalloc, whose image lives in
its fixed control block."""
import numpy as np
import pytest

import oracle
import paper_1801_05857_amd as gx
import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

# Each image holds at least one offsets array of n_states + 1 words per
# process, so these exceed 11776 words (46 KiB) by construction:
#   4 x 4097, 3 x 4097 and 8193 + 8192 x 2 targets (live states) words.
CASES = {
    "four_procs_4096_declared": lambda: W.random_lts(21, 4, 4096, 12, 3, 32, 0.25, 0.1),
    "two_words_4096_declared": lambda: W.random_lts(23, 3, 4096, 16, 3, 32, 0.25, 0.1),
    "one_8192_state_process": lambda: W.random_lts(22, 3, [8192, 32, 32], [8192, 20, 20], 2, 16,
                                                   0.25, 0.05),
    "two_large_processes": lambda: W.random_lts(24, 2, [8192, 8192], [6000, 300], 2, 16, 0.25,
                                                0.02),
}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dedup", [False, True])
def test_large_image_matches_oracle(dev, name, dedup):
    net = CASES[name]()
    want = oracle.explore(net, want_visited=True)
    w = gx.network_words(net)
    with gx.Table(w, 16, max(64, 2 * want.n_states), subgroup=4, max_hashes=32) as t:
        for _ in range(2):  # the second run reuses the table's image buffer
            t.clear()
            got = gx.explore(net, t, local_dedup=dedup)
            assert got.n_states == want.n_states
            assert got.levels.tolist() == want.levels.tolist()
            assert got.n_transitions == want.n_transitions
            assert np.array_equal(got.deadlocks, want.deadlocks)
        assert np.array_equal(t.dump(), want.visited)


def test_small_and_large_images_alternate_in_one_table(dev):
    """One table explores a large-image network (global image, no small-level
    path), a small-image one (LDS image, small levels on one workgroup) and
    the large one again."""
    large = CASES["four_procs_4096_declared"]()
    small = W.random_lts(5, 3, 2048, 12, 3, 32, 0.25, 0.1)  # 3 x 2049 offsets: fits LDS
    assert gx.network_words(small) == gx.network_words(large) == 2
    want = {id(large): oracle.explore(large, want_visited=True),
            id(small): oracle.explore(small, want_visited=True)}
    with gx.Table(2, 16, 1 << 16, subgroup=4, max_hashes=32) as t:
        for net in (large, small, large):
            t.clear()
            got = gx.explore(net, t)
            ref = want[id(net)]
            assert got.levels.tolist() == ref.levels.tolist()
            assert got.n_transitions == ref.n_transitions
            assert np.array_equal(got.deadlocks, ref.deadlocks)
            assert np.array_equal(t.dump(), ref.visited)


def test_batch_server_and_noalloc_refuse_large_images(dev):
    net = CASES["four_procs_4096_declared"]()
    with pytest.raises(gx.GxError) as e:
        gx.explore_batch([net], [1 << 16])
    assert e.value.code == gx.GX_EINVAL
    with gx.Server(1 << 30) as s:
        with pytest.raises(gx.GxError) as e:
            s.submit(net, 1 << 15)
        assert e.value.code == gx.GX_EINVAL
    with gx.Table(2, 16, 1 << 16, subgroup=4) as t:
        with pytest.raises(gx.GxError) as e:
            gx.explore_noalloc(net, t)
        assert e.value.code == gx.GX_EINVAL
