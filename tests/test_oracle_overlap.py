"""Pins for the overlap operator of Eq. (1) and the CGNR solver on it.

* Dov^dag as the oracle forms it (sgn of gamma5 Dw(-mu) after gamma5) is the
  conjugate transpose of the dense Dov (checks the adjoint of the sign and
  where gamma5 sits).
* Ginsparg-Wilson: gamma5 Dov + Dov gamma5 = Dov gamma5 Dov (follows from
  sgn^2 = 1, at any mu).
* At mu = 0, Dov = 1 + (unitary) is normal with its spectrum on the circle
  |z - 1| = 1.
* CGNR reaches np.linalg.solve's solution; on a diagonal matrix with three
  distinct moduli it terminates in three iterations (CG on the normal
  equations has only three distinct eigenvalues to resolve).
"""
import numpy as np
import pytest

import latgen
from oracle import dense as D
from oracle import overlap as O
from oracle import wilson as W

M_W = -1.0


@pytest.fixture(scope="module", params=[0.0, 0.3])
def ov(request):
    mu = request.param
    dims = (2, 2, 4, 4)
    u = latgen.random_gauge(dims, 0.8, 0)
    x = latgen.random_sources(dims, 2, 1)
    s_plus = D.sign_schur(W.dense_matrix(u, M_W, mu))
    s_minus = D.sign_schur(W.dense_matrix(u, M_W, -mu))
    return mu, x, s_plus, s_minus


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_apply_matches_dense(ov):
    mu, x, sp, sm = ov
    v = x[0]
    y = O.dov_apply(lambda w: (sp @ w.reshape(-1)).reshape(w.shape), v)
    assert _rel(y, O.dense_dov(sp) @ v.reshape(-1)) < 1e-13


def test_dagger_is_the_adjoint(ov):
    mu, x, sp, sm = ov
    v = x[0]
    y = O.dov_dag_apply(lambda w: (sm @ w.reshape(-1)).reshape(w.shape), v)
    assert _rel(y, O.dense_dov(sp).conj().T @ v.reshape(-1)) < 1e-11


def test_ginsparg_wilson(ov):
    mu, x, sp, sm = ov
    d = O.dense_dov(sp)
    g = np.diag(np.tile(np.repeat(O.G5, 3), d.shape[0] // 12))
    lhs = g @ d + d @ g
    assert np.linalg.norm(lhs - d @ g @ d) < 1e-11 * np.linalg.norm(lhs)


def test_spectrum_on_circle_at_mu0(ov):
    mu, x, sp, sm = ov
    if mu != 0.0:
        pytest.skip("the circle holds for the Hermitian case")
    ev = np.linalg.eigvals(O.dense_dov(sp))
    assert np.max(np.abs(np.abs(ev - 1.0) - 1.0)) < 1e-11


def test_cgnr_reaches_the_dense_solution(ov):
    mu, x, sp, sm = ov
    d = O.dense_dov(sp)
    b = x[1].reshape(-1)
    y, it, res, hist = O.cgnr(lambda v: d @ v, lambda v: d.conj().T @ v, b, 1e-12, 200)
    assert res <= 1e-12 and it < 40
    assert _rel(y, np.linalg.solve(d, b)) < 1e-11
    assert _rel(d @ y, b) < 2e-12


def test_cgnr_terminates_on_three_distinct_moduli():
    rng = np.random.default_rng(0)
    mods = np.repeat([0.5, 1.0, 2.0], 20)
    d = mods * np.exp(1j * rng.uniform(0, 2 * np.pi, mods.size))
    b = rng.normal(size=mods.size) + 1j * rng.normal(size=mods.size)
    y, it, res, hist = O.cgnr(lambda v: d * v, lambda v: d.conj() * v, b, 1e-12, 10)
    assert it == 3
    assert hist[2] > 1e-3  # not done before the third step
    assert _rel(y, b / d) < 1e-12


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_adjoint_deflation_swaps_left_and_right(mu):
    """A^dag has the eigenvalues conj(lambda), right eigenvectors L and left
    eigenvectors R: deflating every eigenpair of A^dag that way gives its
    spectral sign, i.e. the sign inside Dov^dag."""
    from oracle import deflation as F

    dims = (2, 2, 2, 2)
    u = latgen.random_gauge(dims, 1.0, 3)
    x = latgen.random_sources(dims, 1, 3)[0]
    a = W.dense_matrix(u, M_W, mu)
    ad = W.dense_matrix(u, M_W, -mu)
    assert np.array_equal(ad, a.conj().T)
    lam, r, l = F.critical_eigenpairs(a, a.shape[0], mu == 0.0)
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, mu).reshape(-1)
    y, _ = F.deflated_sign_apply(f, fd, x, 8, 0, mu == 0.0, lam.conj(), l, r)
    assert _rel(y, D.sign_schur(ad) @ x.reshape(-1)) < 1e-11
