"""Step-level GPU parity of the outer Krylov recurrences (Sec. 2).

The first 30 coefficients (alpha, beta, delta) of Lanczos (mu = 0) and
two-sided Lanczos (mu = 0.3) agree with the oracle to 1e-12 relative: both
sides compute the same recurrence in FP64, and over 30 steps rounding
differences between GPU tree reductions and numpy's sums stay far below that.
At the full 16^4 size the coefficients are checked against the oracle run
on the same input for the first steps.
"""
import numpy as np
import pytest

import latgen
from oracle import nested as N
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, make_lattice, nk, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_coefs(u, x, mu, k):
    shape = x.shape
    f = lambda v: W.a_apply(u, v.reshape(shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(shape), M_W, -mu).reshape(-1)
    kr = N.outer_basis(f, fd, x.reshape(-1), k, mu == 0.0)
    return kr.H


@pytest.mark.parametrize("dims,eps", [((4, 4, 4, 4), 0.6), ((2, 4, 6, 8), 0.8), ((16, 16, 16, 16), 0.8)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_first_coefficients_match(dims, eps, mu):
    k = 30 if dims[0] < 16 else 8
    banner(f"basis coefficients dims={dims} eps={eps} mu={mu} k={k}")
    lat, u = make_lattice(dims, eps, seed=0)
    b = nk()
    x = latgen.random_sources(dims, 1, 0)[0]
    p = b.nk_sign_params_default(k=k, mu=mu, m_w=M_W)
    a, be, de, info, rc = b.nk_krylov_basis_device(lat.h, p, to_dev(x))
    torch_cuda().cuda.synchronize()
    assert rc == 0 and info.k_used == k
    H = _oracle_coefs(u, x, mu, k)
    scale = np.max(np.abs(H.alpha))
    assert np.max(np.abs(a - H.alpha)) < 1e-12 * scale
    assert np.max(np.abs(be[: k - 1] - H.beta)) < 1e-12 * scale
    assert np.max(np.abs(de[: k - 1] - H.delta)) < 1e-12 * scale
    if mu == 0.0:
        assert np.all(a.imag == 0) and np.allclose(be, de)
    lat.close()


def test_fp32_coefficients_close():
    dims = (4, 4, 4, 4)
    mu = 0.3
    banner("FP32 / BF16-link basis coefficients vs FP64 oracle")
    lat, u = make_lattice(dims, 0.6, seed=0)
    b = nk()
    x = latgen.random_sources(dims, 1, 0)[0]
    H = _oracle_coefs(u, x, mu, 10)
    for prec, tol in ((b.NK_PREC_FP32, 1e-5), (b.NK_PREC_FP32_BF16LINKS, 5e-2)):
        p = b.nk_sign_params_default(k=10, mu=mu, precision=prec)
        a, be, de, info, rc = b.nk_krylov_basis_device(lat.h, p, to_dev(x))
        scale = np.max(np.abs(H.alpha))
        assert np.max(np.abs(a - H.alpha)) < tol * scale, prec
    lat.close()


def test_zero_source_is_an_error():
    dims = (2, 2, 2, 2)
    lat, _ = make_lattice(dims, 0.5)
    b = nk()
    for mu in (0.0, 0.3):
        p = b.nk_sign_params_default(k=5, mu=mu)
        with pytest.raises(b.NKError) as ei:
            b.nk_krylov_basis_device(lat.h, p, to_dev(np.zeros(12 * 16, np.complex128)))
        assert ei.value.code == b.NK_EINVAL
    lat.close()
