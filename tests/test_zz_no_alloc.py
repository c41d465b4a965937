"""nk_apply_dw_noalloc_device (for callers that cannot allocate): the operator with its temporaries in the
library's fixed device array, against nk_apply_dw_device (bit for bit), on
two calls in a row, the second on a smaller lattice (the device's free
memory before and after is printed); and the size limit."""
import numpy as np
import pytest

import latgen
from tests.gpu_helpers import M_W, banner, make_lattice, nk, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _pair(lat, dims, nrhs, mu, g5, seed):
    b = nk()
    torch = torch_cuda()
    x = to_dev(latgen.random_sources(dims, nrhs, seed))
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, float("nan"))
    b.nk_apply_dw_device(lat.h, M_W, mu, g5, x, y_ref, nrhs)
    b.nk_apply_dw_noalloc_device(lat.h, M_W, mu, g5, x, y_na, nrhs)
    torch.cuda.synchronize()
    return to_host(y_ref), to_host(y_na)


def test_noalloc_matches_allocating_entry_point():
    b = nk()
    torch = torch_cuda()
    big, small = (16, 16, 16, 16), (8, 4, 4, 8)
    lat1, _ = make_lattice(big, 0.8, seed=0)
    lat2, _ = make_lattice(small, 0.6, seed=1)
    # warm both entry points once (the allocating one sizes its handle
    # workspace; the fixed array's code object is loaded on first use)
    _pair(lat1, big, 1, 0.3, True, 20)
    _pair(lat2, small, 1, 0.3, True, 21)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    banner("no-alloc apply: 16^4, 2 sources, mu=0.3, gamma5")
    r1, n1 = _pair(lat1, big, 2, 0.3, True, 22)
    banner("no-alloc apply: 8x4x4x8, 3 sources, mu=0, no gamma5 (smaller, second call)")
    r2, n2 = _pair(lat2, small, 3, 0.0, False, 23)
    free1 = torch.cuda.mem_get_info()[0]
    assert np.array_equal(n1.view(np.uint64), r1.view(np.uint64))
    assert np.array_equal(n2.view(np.uint64), r2.view(np.uint64))
    assert np.isfinite(n1).all() and np.isfinite(n2).all()
    print(f"[no-alloc] free device memory before/after the measured calls: {free0} / {free1}", flush=True)
    lat1.close()
    lat2.close()


def test_noalloc_rejects_lattices_beyond_its_workspace():
    b = nk()
    torch = torch_cuda()
    dims = (16, 16, 16, 32)
    lat, _ = make_lattice(dims, 0.0, unit=True)
    n = 12 * 16 * 16 * 16 * 32
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(b.NKError) as ei:
        b.nk_apply_dw_noalloc_device(lat.h, M_W, 0.3, True, x, y)
    assert ei.value.code == b.NK_EINVAL
    assert "exceed" in b.nk_last_error()
    lat.close()
