"""The measurement probes behind the roofline's ceilings (gx_gather_probe,
gx_claim_probe) run and touch what they should."""
import pytest

import paper_1801_05857_amd as gx

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gx.lib()
    return torch.device("cuda:0")


def test_gather_probe_sums_what_it_reads(dev):
    buf = torch.ones(1 << 20, dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    gx.gather_probe(buf, 64, 4096, 7, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 4096 * 16  # 16 lanes read 1 each per 64-byte read


@pytest.mark.parametrize("mode", [1, 2])
def test_claim_probe_claims_words(dev, mode):
    buf = torch.full((1 << 20,), -1, dtype=torch.int64, device=dev)  # 131072 granules
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    gx.claim_probe(buf, mode, 4096, 7, sink)
    torch.cuda.synchronize()
    g = buf.view(-1, 8).cpu()
    assert (g[:, 0] == -1).all()          # the word read is never claimed
    assert (g[:, 3:] == -1).all()         # nor any past the two claim words
    claimed = int((g[:, 1:3] != -1).sum())
    # mode 1: every operation claims, mode 2 every other one; a granule drawn
    # twice keeps its first claim (about 1.6% of 4096 draws over 131072)
    want = 4096 if mode == 1 else 2048
    assert 0.95 * want <= claimed <= want
    assert ((g[:, 1:3] == -1) | (g[:, 1:3] % 2 == 1)).all()  # claims write odd values
