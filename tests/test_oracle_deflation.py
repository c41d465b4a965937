"""Pins for the deflated sign (Sec. 2, exact treatment of critical eigenvalues).

* The eigenpairs satisfy their definitions: A R = R Lambda, L^dag A = Lambda L^dag,
  L^dag R = I, and they are the ones with the smallest |Re lambda|.
* Deflating every eigenpair leaves nothing for the Krylov part, and the result
  is the spectral sign of Eq. (2) written with the dense eigen-decomposition.
* A source in the span of deflated eigenvectors: sgn(A) r_i = sgn(Re lambda_i) r_i.
* The projected source has no component along the deflated right eigenvectors
  as seen by the left ones (L^dag x' = 0).
* m = 0 is the Krylov method itself, bit for bit.
* Deflating the critical eigenvalues at fixed k makes the approximation more
  accurate, the reason the paper gives for it.
"""
import numpy as np
import pytest

import latgen
from oracle import deflation as F
from oracle import dense as D
from oracle import nested as N
from oracle import wilson as W

M_W = -1.0


def _setup(dims, mu, eps=0.8, seed=0):
    u = latgen.random_gauge(dims, eps, seed)
    x = latgen.random_sources(dims, 1, seed)[0]
    shape = x.shape
    f = lambda v: W.a_apply(u, v.reshape(shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(shape), M_W, -mu).reshape(-1)
    a = W.dense_matrix(u, M_W, mu)
    return a, x, f, fd


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.fixture(scope="module", params=[0.0, 0.3])
def case(request):
    mu = request.param
    a, x, f, fd = _setup((2, 2, 4, 4), mu)
    herm = mu == 0.0
    lam, r, l = F.critical_eigenpairs(a, 16, herm)
    exact = D.sign_spectral(a, hermitian=herm) @ x.reshape(-1)
    return mu, a, x, f, fd, lam, r, l, exact


def test_eigenpairs_satisfy_their_definitions(case):
    mu, a, x, f, fd, lam, r, l, exact = case
    na = np.linalg.norm(a, 2)
    assert np.linalg.norm(a @ r - r * lam) < 1e-11 * na
    assert np.linalg.norm(l.conj().T @ a - lam[:, None] * l.conj().T) < 1e-10 * na * np.linalg.norm(l, 2)
    assert np.linalg.norm(l.conj().T @ r - np.eye(len(lam))) < 1e-10
    # they are the critical ones: no other eigenvalue is closer to the imaginary axis
    rest = np.linalg.eigvals(a)
    assert np.abs(lam.real).max() <= np.sort(np.abs(rest.real))[len(lam) - 1] + 1e-10


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_deflation_is_the_spectral_sign(mu):
    a, x, f, fd = _setup((2, 2, 2, 2), mu, eps=1.0, seed=3)
    herm = mu == 0.0
    n = a.shape[0]
    lam, r, l = F.critical_eigenpairs(a, n, herm)
    y, info = F.deflated_sign_apply(f, fd, x, 8, 0, herm, lam, r, l)
    assert info["projected_norm"] < 1e-12 * np.linalg.norm(x)
    ref = D.sign_schur(a) @ x.reshape(-1)
    assert _rel(y, ref) < 1e-11


def test_source_in_deflated_span(case):
    mu, a, x, f, fd, lam, r, l, exact = case
    herm = mu == 0.0
    xs = (r[:, 0] + 0.5j * r[:, 3]).reshape(x.shape)
    y, info = F.deflated_sign_apply(f, fd, xs, 20, 10, herm, lam, r, l)
    s = np.sign(lam.real)
    ref = s[0] * r[:, 0] + 0.5j * s[3] * r[:, 3]
    assert info["projected_norm"] < 1e-12 * np.linalg.norm(xs)
    assert _rel(y, ref) < 1e-11


def test_projected_source_is_free_of_deflated_modes(case):
    mu, a, x, f, fd, lam, r, l, exact = case
    c, xp = F.project(x.reshape(-1), r, l)
    assert np.linalg.norm(l.conj().T @ xp) < 1e-12 * np.linalg.norm(x)
    # and the exact part is f(A) applied to R c
    sa = D.sign_spectral(a, hermitian=mu == 0.0)
    assert _rel(r @ (F.sgn(lam) * c), sa @ (r @ c)) < 1e-11


def test_no_deflation_is_the_krylov_method(case):
    mu, a, x, f, fd, lam, r, l, exact = case
    herm = mu == 0.0
    y0, _ = N.sign_apply(f, fd, x, 60, 30, herm)
    y1, _ = F.deflated_sign_apply(f, fd, x, 60, 30, herm, lam[:0], r[:, :0], l[:, :0])
    assert np.array_equal(y0, y1)


@pytest.mark.parametrize("ell", [0, 40])
def test_deflation_improves_accuracy_at_fixed_k(case, ell):
    mu, a, x, f, fd, lam, r, l, exact = case
    herm = mu == 0.0
    y0, _ = N.sign_apply(f, fd, x, 80, ell, herm)
    yd, _ = F.deflated_sign_apply(f, fd, x, 80, ell, herm, lam, r, l)
    e0, ed = _rel(y0, exact), _rel(yd, exact)
    assert ed < e0 / 10, (e0, ed)


def test_sign_undefined_on_the_imaginary_axis():
    with pytest.raises(ValueError):
        F.sgn(np.array([0.5 + 0j, 2j]))
