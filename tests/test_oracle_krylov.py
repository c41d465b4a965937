"""Pins for the Lanczos and two-sided Lanczos bases (Sec. 2, Eq. (3)).

Checks the defining properties the paper states: V_k orthonormal and
H_k = V_k^dag A V_k (Hermitian), W_k^dag V_k = 1 and H_k = W_k^dag A V_k
(two-sided), H_k tridiagonal, and exact termination: with full
re-(bi)orthogonalisation at k = n the Ritz approximation equals the exact
spectral sign.
"""
import numpy as np
import pytest

import latgen
from oracle import dense as D
from oracle import krylov as K
from oracle import nested as N
from oracle import wilson as W

M_W = -1.0


def _setup(dims, mu, eps=0.8, seed=0):
    u = latgen.random_gauge(dims, eps, seed)
    x = latgen.random_sources(dims, 1, seed)[0]
    shape = x.shape
    f = lambda v: W.a_apply(u, v.reshape(shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(shape), M_W, -mu).reshape(-1)
    return u, x, f, fd


def test_lanczos_relations():
    u, x, f, _ = _setup((4, 4, 2, 4), 0.0)
    kr = K.lanczos(f, x, 30)
    V = kr.V
    assert np.linalg.norm(V.conj().T @ V - np.eye(30)) < 1e-10
    AV = np.stack([f(V[:, j]) for j in range(30)], axis=1)
    assert np.linalg.norm(V.conj().T @ AV - kr.H.dense()) < 1e-10
    assert np.allclose(kr.H.alpha.imag, 0) and np.allclose(kr.H.beta, kr.H.delta)


def test_two_sided_relations():
    u, x, f, fd = _setup((4, 4, 2, 4), 0.3)
    kr = K.two_sided_lanczos(f, fd, x, 30)
    V, Wm = kr.V, kr.W
    assert np.linalg.norm(Wm.conj().T @ V - np.eye(30)) < 1e-9
    AV = np.stack([f(V[:, j]) for j in range(30)], axis=1)
    assert np.linalg.norm(Wm.conj().T @ AV - kr.H.dense()) < 1e-9 * np.linalg.norm(kr.H.dense())
    # the Krylov relation A V_k = V_k H_k + delta_{k+1} v_{k+1} e_k^T holds on all but the last column
    r = AV[:, :-1] - V @ kr.H.dense()[:, :-1]
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(AV)


def test_two_sided_reduces_to_lanczos_at_mu_zero():
    u, x, f, fd = _setup((2, 2, 4, 4), 0.0)
    a = K.lanczos(f, x, 20)
    b = K.two_sided_lanczos(f, fd, x, 20)
    assert np.allclose(a.H.alpha, b.H.alpha, atol=1e-12)
    assert np.allclose(a.H.beta, b.H.beta, atol=1e-12)
    assert np.allclose(a.H.beta, b.H.delta, atol=1e-12)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_exact_termination(mu):
    dims = (2, 2, 2, 2)
    u, x, f, fd = _setup(dims, mu)
    a = W.dense_matrix(u, M_W, mu)
    n = a.shape[0]
    kr = N.outer_basis(f, fd, x.reshape(-1), n, mu == 0.0, reorth=True)
    assert kr.breakdown == 0
    z, _ = N.small_sign(kr.H, 0, mu == 0.0)
    y = kr.norm_x * kr.V @ z
    ref = D.sign_spectral(a) @ x.reshape(-1)
    assert np.linalg.norm(y - ref) < 1e-10 * np.linalg.norm(ref)


def test_serious_breakdown_detected():
    # v1 = w1 = e1; A v1 = (1, 1, 0), A^dag w1 = (1, 0, 1): after removing the
    # alpha term the two new directions are orthogonal although neither is zero.
    a = np.array([[1, 0, 1], [1, 2, 0], [0, 0, 3]], dtype=np.complex128)
    x = np.array([1, 0, 0], dtype=np.complex128)
    kr = K.two_sided_lanczos(lambda v: a @ v, lambda w: a.conj().T @ w, x, 3)
    assert kr.breakdown == 1
    assert kr.H.k == 1


def test_dense_tridiagonal_layout():
    t = K.Tridiag(np.array([1.0, 2.0, 3.0]), np.array([4.0, 5.0]), np.array([6.0, 7.0]))
    h = t.dense()
    assert h[0, 1] == 4.0 and h[1, 0] == 6.0 and h[2, 1] == 7.0 and h[1, 2] == 5.0
    assert np.count_nonzero(h) == 7


@pytest.mark.parametrize("mu", [0.3, 0.5])
def test_serious_breakdown_on_a_free_field_plane_wave(mu):
    """The lattice operator itself: a plane wave times a spinor with
    w_hat^dag v_hat = 0 (tests/breakdown_source.py) stops the oracle's 2sL
    after one step, while v_hat and w_hat are far from zero."""
    from tests import breakdown_source as B

    s, r = B.breakdown_spinor(M_W, mu)
    assert r < 1e-14
    M = B.momentum_matrix(M_W, mu)
    a = s.conj() @ M @ s
    assert np.linalg.norm(M @ s - a * s) > 0.1  # not an eigenvector
    x = B.plane_wave(s)
    u = latgen.unit_gauge(B.DIMS)
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -mu).reshape(-1)
    # the plane wave stays in its four spinor directions at p
    assert np.linalg.norm(f(x.reshape(-1)) - B.plane_wave(M @ s).reshape(-1)) < 1e-13
    kr = K.two_sided_lanczos(f, fd, x.reshape(-1), 10)
    assert kr.breakdown == 1
    assert kr.H.k == 1
    assert abs(kr.H.alpha[0] - a) < 1e-13
