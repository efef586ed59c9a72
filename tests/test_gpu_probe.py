"""The HBM streaming probe (gpe_hbm_stream, the bandwidth reference of the
roofline figures) moves exactly the bytes it is asked to: a copy reproduces
its source bitwise, a write fills its destination with 1.0, a read leaves
the destination as it was, with the default and explicit work-group counts
and a ragged element count."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes,wg", [(16 * 1000003, 0), (16 * 4099, 7), (16, 1)])
def test_stream_probe_moves_the_bytes(nbytes, wg):
    import torch

    from paper_2011_00814_amd import gpe as G

    G.lib()
    n = nbytes // 4
    rng = np.random.default_rng(5)
    src = torch.tensor(rng.normal(size=n).astype(np.float32), device="cuda:0")
    dst = torch.full((n,), -3.0, dtype=torch.float32, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    G.gpe_hbm_stream(G.GPE_STREAM_READ, dst.data_ptr(), src.data_ptr(), nbytes, wg, s)
    torch.cuda.synchronize()
    assert bool(torch.all(dst == -3.0))
    G.gpe_hbm_stream(G.GPE_STREAM_COPY, dst.data_ptr(), src.data_ptr(), nbytes, wg, s)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    G.gpe_hbm_stream(G.GPE_STREAM_WRITE, dst.data_ptr(), src.data_ptr(), nbytes, wg, s)
    torch.cuda.synchronize()
    assert bool(torch.all(dst == 1.0))
