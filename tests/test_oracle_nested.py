"""Pins for the non-nested and nested approximations (Eqs. (3), (5), (6)).

* Eq. (6) on the Ritz matrix: sgn(H_k) e1 = sgn(H_k + H_k^{-1}) e1 (dense eig).
* Naive nesting (Sec. 3): the inner space K_l(H_k, e1) only sees the leading
  l x l block of H_k, so the unpreconditioned nested result equals
  [sgn(H_l) e1; 0] -- the non-nested result at k = l.
* l = k: the nested result equals the non-nested one.
* End to end against the exact spectral sign (Eq. (2)), sgn^2 = 1, and the
  Ginsparg-Wilson relation of Dov = 1 + gamma5 sgn(gamma5 Dw) (Eq. (1)).
* The paper's soft claims: l << k loses nothing (Sec. 4), and the
  preconditioning improves the condition number (Sec. 3).
"""
import numpy as np
import pytest

import latgen
from oracle import dense as D
from oracle import krylov as K
from oracle import nested as N
from oracle import wilson as W

M_W = -1.0


def _op(dims, mu, eps, seed=0):
    u = latgen.random_gauge(dims, eps, seed)
    x = latgen.random_sources(dims, 1, seed)[0]
    shape = x.shape
    f = lambda v: W.a_apply(u, v.reshape(shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(shape), M_W, -mu).reshape(-1)
    return u, x, f, fd


@pytest.fixture(scope="module", params=[0.0, 0.3])
def basis(request):
    mu = request.param
    u, x, f, fd = _op((4, 4, 4, 4), mu, 0.6)
    kr = N.outer_basis(f, fd, x.reshape(-1), 120, mu == 0.0)
    return mu, u, x, kr


def test_eq6_on_ritz_matrix(basis):
    mu, u, x, kr = basis
    h = kr.H.dense()
    s1 = D.sign_spectral(h, hermitian=False)[:, 0]
    s2 = D.sign_spectral(h + np.linalg.inv(h), hermitian=False)[:, 0]
    assert np.linalg.norm(s1 - s2) < 1e-10 * np.linalg.norm(s1)
    # and RH on H_k reproduces the spectral vector
    z, _ = N.small_sign(kr.H, 0, mu == 0.0)
    assert np.linalg.norm(z - s1) < 1e-10 * np.linalg.norm(s1)


def test_naive_nesting_sees_leading_block(basis):
    mu, u, x, kr = basis
    herm = mu == 0.0
    for ell in (10, 37, 80):
        zn, _ = N.small_sign(kr.H, ell, herm, precondition=False)
        zl, _ = N.small_sign(kr.H.leading(ell), 0, herm)
        ref = np.zeros_like(zn)
        ref[:ell] = zl
        assert np.linalg.norm(zn - ref) < 1e-10 * np.linalg.norm(ref)


def test_full_inner_space_equals_nonnested(basis):
    mu, u, x, kr = basis
    herm = mu == 0.0
    z0, _ = N.small_sign(kr.H, 0, herm)
    zk, _ = N.small_sign(kr.H, kr.H.k, herm)
    assert np.linalg.norm(z0 - zk) < 1e-9 * np.linalg.norm(z0)


def test_preconditioning_improves_conditioning(basis):
    mu, u, x, kr = basis
    h = kr.H.dense()
    b = h + np.linalg.inv(h)
    assert np.linalg.cond(b) < np.linalg.cond(h)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_nested_vs_exact_tiny(mu):
    dims = (2, 2, 2, 4)
    u, x, f, fd = _op(dims, mu, 0.2)
    ref = D.sign_spectral(W.dense_matrix(u, M_W, mu)) @ x.reshape(-1)
    y, info = N.sign_apply(f, fd, x, 150, 60, mu == 0.0)
    tol = 1e-9 if mu == 0.0 else 1e-7
    assert np.linalg.norm(y.reshape(-1) - ref) < tol * np.linalg.norm(ref)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_sign_squared_is_identity(mu):
    dims = (2, 2, 4, 4)
    u, x, f, fd = _op(dims, mu, 0.2)
    y, _ = N.sign_apply(f, fd, x, 200, 80, mu == 0.0)
    yy, _ = N.sign_apply(f, fd, y, 200, 80, mu == 0.0)
    tol = 1e-8 if mu == 0.0 else 1e-6
    assert np.linalg.norm(yy - x) < tol * np.linalg.norm(x)
    if mu == 0.0:
        assert abs(np.linalg.norm(y) - np.linalg.norm(x)) < tol * np.linalg.norm(x)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_ginsparg_wilson(mu):
    # Dov = 1 + g5 eps with eps^2 = 1 obeys g5 D + D g5 = D g5 D.
    dims = (2, 2, 2, 4)
    u, x, f, fd = _op(dims, mu, 0.2)
    g5 = np.kron(np.eye(dims[0] * dims[1] * dims[2] * dims[3]), np.kron(W.gamma5(), np.eye(3)))

    def sgn(v):
        y, _ = N.sign_apply(f, fd, v.reshape(x.shape), 200, 80, mu == 0.0)
        return y.reshape(-1)

    def dov(v):
        return v + g5 @ sgn(v)

    v = x.reshape(-1)
    lhs = g5 @ dov(v) + dov(g5 @ v)
    rhs = dov(g5 @ dov(v))
    tol = 1e-8 if mu == 0.0 else 1e-6
    assert np.linalg.norm(lhs - rhs) < tol * np.linalg.norm(lhs)


def test_config1_plain_and_nested_vs_full_eig():
    # 4^4, mu = 0, eps = 0.4, k = 150; nested l = 60; the full-eig result is
    # stored by tests/golden/make_golden.py (oracle.dense.sign_spectral)
    import os

    dims = (4, 4, 4, 4)
    u, x, f, fd = _op(dims, 0.0, 0.4)
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_4x4x4x4_mu0_eps0.4.npy")
    ref = np.load(gold)
    yp, _ = N.sign_apply(f, fd, x, 150, 0, True)
    yn, _ = N.sign_apply(f, fd, x, 150, 60, True)
    ep = np.linalg.norm(yp.reshape(-1) - ref) / np.linalg.norm(ref)
    en = np.linalg.norm(yn.reshape(-1) - ref) / np.linalg.norm(ref)
    assert ep < 1e-7
    # no loss of accuracy at l = 60 << k = 150 (Sec. 4)
    assert en < 1.5 * ep


def test_convergence_estimate_sanity(basis):
    mu, u, x, kr = basis
    herm = mu == 0.0
    est = N.convergence_estimate(kr.H, 0, herm, 10)
    assert 0.0 < est < 1.0


@pytest.mark.parametrize("k,d,ell", [(40, 10, 0), (60, 5, 0), (60, 10, 20), (90, 20, 30), (120, 10, 40)])
def test_convergence_estimate_between_the_true_errors(k, d, ell):
    """The estimate (R15) pinned against the exact sign.  At mu = 0 with a
    fully reorthogonalised Lanczos basis V_k has orthonormal columns, so
    est ||y_k|| = ||y_k - y_{k-d}|| with y_j = ||x|| V_j z^{(j)}; the triangle
    inequality against the exact spectral sign y* (stored 4^4 result) then
    brackets it: |e_{k-d} - e_k| <= est ||y_k|| <= e_{k-d} + e_k, with
    e_j = ||y_j - y*||."""
    import os

    dims = (4, 4, 4, 4)
    u = latgen.random_gauge(dims, 0.4, 0)
    x = latgen.random_sources(dims, 1, 0)[0]
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_4x4x4x4_mu0_eps0.4.npy"))
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, 0.0).reshape(-1)
    kr = K.lanczos(f, x.reshape(-1), k, reorth=True)
    assert np.linalg.norm(kr.V.conj().T @ kr.V - np.eye(kr.V.shape[1])) < 1e-13
    est = N.convergence_estimate(kr.H, ell, True, d)
    z1, _ = N.small_sign(kr.H, ell, True)
    z0, _ = N.small_sign(kr.H.leading(k - d), min(ell, k - d) if ell else 0, True)
    y1 = kr.norm_x * kr.V[:, :k] @ z1
    y0 = kr.norm_x * kr.V[:, : k - d] @ z0
    e1, e0, n1 = np.linalg.norm(y1 - ref), np.linalg.norm(y0 - ref), np.linalg.norm(y1)
    slack = 1e-12 * n1
    assert abs(e0 - e1) - slack <= est * n1 <= e0 + e1 + slack


def _ritz(mu, k):
    u, x, f, fd = _op((4, 4, 4, 4), mu, 0.6)
    return N.outer_basis(f, fd, x.reshape(-1), k, mu == 0.0).H


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_arnoldi_relations(mu):
    """The inner Arnoldi option: orthonormal V and H = V^dag B V (upper
    Hessenberg), by matrix products rather than the recurrence."""
    h = _ritz(mu, 80).dense()
    b = h + np.linalg.solve(h, np.eye(h.shape[0]))
    V, H = N.arnoldi(b, 30)
    assert np.linalg.norm(V.conj().T @ V - np.eye(30)) < 1e-13
    assert np.linalg.norm(V.conj().T @ b @ V - H) < 1e-12 * np.linalg.norm(b)
    assert np.count_nonzero(np.tril(H, -2)) == 0


def test_arnoldi_on_hermitian_b_is_lanczos():
    """For Hermitian B the Arnoldi Hessenberg matrix is the Lanczos
    tridiagonal one (two routes to the same H_l)."""
    h = _ritz(0.0, 80).dense()
    b = h + np.linalg.solve(h, np.eye(h.shape[0]))
    _, H = N.arnoldi(b, 30)
    L = N.inner_basis(b, 30, True).H.dense()
    assert np.linalg.norm(H - L) < 1e-11 * np.linalg.norm(L)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_arnoldi_nested_at_full_inner_size_is_non_nested(mu):
    H = _ritz(mu, 60)
    z0, _ = N.small_sign(H, 0, mu == 0.0)
    z1, _ = N.small_sign(H, 60, mu == 0.0, inner="arnoldi")
    assert np.linalg.norm(z1 - z0) < 1e-10 * np.linalg.norm(z0)


def test_arnoldi_nested_against_the_exact_sign():
    """End to end at 4^4, mu = 0.3 (stored exact sign): the Arnoldi inner space
    loses nothing against the plain method at l = 80 < k = 150 (whose error
    is 2e-6 here), and agrees with the two-sided inner space to that error."""
    import os

    dims = (4, 4, 4, 4)
    u = latgen.random_gauge(dims, 0.4, 0)
    x = latgen.random_sources(dims, 1, 0)[0]
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_4x4x4x4_mu0.3_eps0.4.npy"))
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, 0.3).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -0.3).reshape(-1)
    yp, _ = N.sign_apply(f, fd, x, 150, 0, False)
    ya, _ = N.sign_apply(f, fd, x, 150, 80, False, inner="arnoldi")
    ys, _ = N.sign_apply(f, fd, x, 150, 80, False)
    ep = np.linalg.norm(yp.reshape(-1) - ref) / np.linalg.norm(ref)
    ea = np.linalg.norm(ya.reshape(-1) - ref) / np.linalg.norm(ref)
    assert ep < 1e-5
    assert ea < 2.0 * ep
    assert np.linalg.norm(ya - ys) < 2.0 * ep * np.linalg.norm(ys)
