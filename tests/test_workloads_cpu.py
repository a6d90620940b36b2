"""The seeded input generators: the device (torch) key streams equal the
numpy ones, and the served request pool has the shape it declares."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n_distinct,dup,w", [(1 << 12, 2, 2), (1 << 12, 2, 1), (1000, 21, 1),
                                              (4096 // 50, 50, 1), (777, 3, 2), (1, 100, 1)])
def test_torch_stream_equals_numpy(n_distinct, dup, w):
    keys, idx = W.duplicated_stream_torch(n_distinct, dup, 1801058570, "cpu", w=w)
    ref = W.duplicated_stream(n_distinct, dup, w, 1801058570)
    assert np.array_equal(keys.numpy().view(np.uint32), ref)
    # every distinct key exactly dup times
    counts = np.bincount(idx.numpy(), minlength=n_distinct)
    assert (counts == dup).all()


def test_served_pool_shape():
    nets, targets, bounds = W.served_networks(256, 5)
    import oracle

    words = [oracle.pack_plan(n.n_states)[0] for n in nets]
    assert set(words) == {1, 2, 3, 4}
    t = np.log10(np.asarray(targets, dtype=np.float64))
    assert t.min() >= 4.0 and t.max() <= 8.0
    # bounds: products of live counts, within a factor of 64 below 2T
    for b, tg in zip(bounds, targets):
        assert b <= 2 * tg + 1 and b * 64 >= 2 * tg
