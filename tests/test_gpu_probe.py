"""The HBM stream probe moves the data it claims to (copy is exact, the mix
is a + 2c in FP32, a ragged size uses every element) and rejects bad
arguments."""
import pytest

pytestmark = pytest.mark.gpu


def test_stream_probe_results_and_errors():
    import torch
    from paper_2008_11778_amd._lib import AafwiError, _lib, stream_probe
    n = 1_000_003 * 4  # 16-byte pieces, not a multiple of the grid
    g = torch.Generator(device="cuda").manual_seed(7)
    a = torch.randn(n, device="cuda", generator=g)
    c = torch.randn(n, device="cuda", generator=g)
    b = torch.zeros(n, device="cuda")
    stream_probe(2, a, b, blocks_per_cu=4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    stream_probe(3, a, b, c, blocks_per_cu=8)
    torch.cuda.synchronize()
    assert torch.equal(b, a + 2.0 * c)
    stream_probe(1, None, b, blocks_per_cu=16)
    torch.cuda.synchronize()
    assert torch.equal(b.view(-1, 4)[-1], torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda"))
    stream_probe(0, a, b)  # reads only
    torch.cuda.synchronize()
    for kind, nbytes, bpc in ((4, 16, 4), (0, 24, 4), (0, 16, 0), (0, 16, 65)):
        with pytest.raises(AafwiError):
            from paper_2008_11778_amd._lib import _check
            _check(_lib.aafwi_stream_probe(None, kind, nbytes, bpc, a.data_ptr(), b.data_ptr(), None))
