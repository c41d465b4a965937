"""Pins for the exact sign (Eq. (2), sgn(z) = sgn(Re z)) and for Eqs. (6)-(7).

The spectral route (eigh/eig) is checked against a Schur-plus-Sylvester route
that uses no eigenvectors, against A (A^2)^{-1/2} for Hermitian A, against the
free-field momentum-space sign, and against the algebraic identities
sgn(A)^2 = 1 and [sgn(A), A] = 0.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import latgen
from oracle import dense as D
from oracle import freefield as F
from oracle import wilson as W

M_W = -1.0
DIMS = (2, 2, 2, 2)


@pytest.fixture(scope="module", params=[0.0, 0.3])
def mat(request):
    mu = request.param
    u = latgen.random_gauge(DIMS, 0.8, 0)
    return mu, W.dense_matrix(u, M_W, mu)


def test_spectral_matches_schur(mat):
    mu, a = mat
    s1 = D.sign_spectral(a)
    s2 = D.sign_schur(a)
    assert np.linalg.norm(s1 - s2) < 1e-12 * np.linalg.norm(s1)


def test_sign_squares_to_one_and_commutes(mat):
    mu, a = mat
    s = D.sign_spectral(a)
    n = a.shape[0]
    assert np.linalg.norm(s @ s - np.eye(n)) < 1e-12 * n
    assert np.linalg.norm(s @ a - a @ s) < 1e-12 * np.linalg.norm(a) * np.sqrt(n)


def test_hermitian_sign_is_polar_factor():
    a = W.dense_matrix(latgen.random_gauge(DIMS, 0.8, 0), M_W, 0.0)
    s = a @ np.linalg.inv(sla.sqrtm(a @ a))
    assert np.linalg.norm(s - D.sign_spectral(a)) < 1e-11 * a.shape[0]


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_sign_matches_dense(mu):
    dims = (2, 2, 2, 4)
    u = latgen.unit_gauge(dims)
    x = latgen.random_sources(dims, 1, 2)[0]
    a = W.dense_matrix(u, M_W, mu)
    y1 = D.sign_spectral(a, hermitian=(mu == 0.0)) @ x.reshape(-1)
    y2 = F.sign_apply_free(x, M_W, mu).reshape(-1)
    assert np.linalg.norm(y1 - y2) < 1e-12 * np.linalg.norm(y1)


def test_sign_of_scalar_multiple_and_eq6():
    rng = np.random.default_rng(3)
    n = 40
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 0.5 * np.eye(n)
    s = D.sign_spectral(a, hermitian=False)
    # Eq. (6): sgn(A) = sgn(A + A^{-1})
    s6 = D.sign_spectral(a + np.linalg.inv(a), hermitian=False)
    assert np.linalg.norm(s - s6) < 1e-10 * np.linalg.norm(s)
    # sgn(c A) = sgn(A) for c > 0
    assert np.linalg.norm(D.sign_spectral(3.7 * a, hermitian=False) - s) < 1e-10 * np.linalg.norm(s)


def test_eq7_scalar_identity():
    rng = np.random.default_rng(5)
    z = rng.standard_normal(10000) + 1j * rng.standard_normal(10000)
    assert np.all(np.sign((z + 1 / z).real) == np.sign(z.real))
