"""The streaming measurement kernels (nk_stream_device) compute what they
claim, so the bandwidth ceiling that bench.py reports comes from real work:
the read-only pass's partial sums add up to |a|^2, the copy is exact, and the
triad is a + b / 2 (exact for these inputs)."""
import numpy as np
import pytest

from tests.gpu_helpers import banner, nk, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,blocks", [(1, 1), (1000, 3), (1 << 20, 256), ((1 << 20) + 7, 1024)])
def test_stream_kernels(n, blocks):
    b = nk()
    torch = torch_cuda()
    banner(f"stream kernels n={n} blocks={blocks}")
    rng = np.random.default_rng(n)
    ah = rng.integers(-8, 8, n) + 1j * rng.integers(-8, 8, n)
    bh = rng.integers(-8, 8, n) + 1j * rng.integers(-8, 8, n)
    a = torch.from_numpy(ah.astype(np.complex128)).to("cuda")
    bb = torch.from_numpy(bh.astype(np.complex128)).to("cuda")
    c = torch.zeros(max(n, blocks), dtype=torch.complex128, device="cuda")
    b.nk_stream_device(0, a, None, c, blocks)
    torch.cuda.synchronize()
    assert float(c[:blocks].real.sum()) == float(np.sum(np.abs(ah) ** 2))
    c = torch.zeros(n, dtype=torch.complex128, device="cuda")
    b.nk_stream_device(1, a, None, c, blocks)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), ah)
    b.nk_stream_device(2, a, bb, c, blocks)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), ah + 0.5 * bh)
    with pytest.raises(b.NKError):
        b.nk_stream_device(3, a, None, c, blocks)
