"""The read-bandwidth probe (a measurement helper): it reads every byte of
the buffer once, so its per-workgroup sums add up to the buffer's sum."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


@pytest.mark.parametrize("n4,blocks,nt", [(250_001, 37, False), (250_001, 4096, True), (1, 1, False),
                                          (3_000_000, 512, False)])
def test_read_probe_reads_every_value(kl, n4, blocks, nt):
    g = torch.Generator(device="cuda").manual_seed(n4 + blocks)
    buf = torch.rand(4 * n4, generator=g, device="cuda")
    out = kl.kmpp_read_probe(buf, blocks=blocks, nontemporal=nt)
    torch.cuda.synchronize()
    want = buf.double().sum().item()
    got = out.double().sum().item()
    assert abs(got - want) <= 1e-5 * want + 1e-6
