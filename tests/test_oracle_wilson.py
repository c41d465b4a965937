"""Pins for the oracle's gamma5 Dw(mu) (Sec. 1, Eq. (1) and the operator it uses).

Each check rests on something other than the oracle's own formula: the
Clifford algebra, the free-field closed form in momentum space,
gamma5-hermiticity (A(mu)^dag = A(-mu), Hermitian at mu = 0), and gauge
covariance.  A few planted mistakes show that the pins catch them.
"""
import numpy as np
import pytest

import latgen
from oracle import freefield as F
from oracle import wilson as W

M_W = -1.0


def test_gamma_clifford_and_gamma5():
    g = W.gamma_matrices()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            anti = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(anti, 2.0 * (a == b) * np.eye(4))
    assert np.allclose(W.gamma5(), np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 4, 2)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_loops_match_vectorised(dims, mu):
    u = latgen.random_gauge(dims, 0.8, 3)
    x = latgen.random_sources(dims, 1, 4)[0]
    a = W.dw_apply(u, x, M_W, mu, g5=True)
    b = W.dw_apply_loops(u, x, M_W, mu, g5=True)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8), (4, 2, 2, 6)])
@pytest.mark.parametrize("mu", [0.0, 0.3, 0.5])
def test_free_field_closed_form(dims, mu):
    x = latgen.random_sources(dims, 1, 11)[0]
    a = W.dw_apply(latgen.unit_gauge(dims), x, M_W, mu, g5=True)
    b = F.g5dw_apply_free(x, M_W, mu)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_gamma5_hermiticity(mu):
    dims = (4, 2, 2, 4)
    u = latgen.random_gauge(dims, 1.0, 5)
    x, y = latgen.random_sources(dims, 2, 6)
    lhs = np.vdot(y, W.a_apply(u, x, M_W, mu))
    rhs = np.vdot(W.a_apply(u, y, M_W, -mu), x)
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs) * 10
    # the term-by-term adjoint agrees with A(-mu)
    d = W.a_dag_apply(u, x, M_W, mu) - W.a_apply(u, x, M_W, -mu)
    assert np.max(np.abs(d)) < 1e-13


def test_hermitian_at_mu_zero_dense():
    dims = (2, 2, 2, 2)
    a = W.dense_matrix(latgen.random_gauge(dims, 0.8, 1), M_W, 0.0)
    assert np.linalg.norm(a - a.conj().T) < 1e-13 * np.linalg.norm(a)
    b = W.dense_matrix(latgen.random_gauge(dims, 0.8, 1), M_W, 0.3)
    assert np.linalg.norm(b - b.conj().T) > 1e-3 * np.linalg.norm(b)


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_gauge_covariance(mu):
    dims = (2, 4, 2, 4)
    u = latgen.random_gauge(dims, 0.9, 2)
    x = latgen.random_sources(dims, 1, 3)[0]
    g = latgen.random_site_su3(dims, 9)
    ug = W.gauge_transform(u, g)
    gx = np.einsum("...ab,...sb->...sa", g, x)
    lhs = W.dw_apply(ug, gx, M_W, mu)
    rhs = np.einsum("...ab,...sb->...sa", g, W.dw_apply(u, x, M_W, mu))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_links_are_su3():
    u = latgen.random_gauge((2, 2, 2, 4), 1.0, 0)
    eye = np.eye(3)
    assert np.max(np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(u) - 1.0)) < 1e-14


# --- planted mistakes: each must be caught by one of the pins above ---------

def _free_field_error(apply):
    dims = (4, 2, 2, 4)
    x = latgen.random_sources(dims, 1, 12)[0]
    a = apply(latgen.unit_gauge(dims), x)
    b = F.g5dw_apply_free(x, M_W, 0.3)
    return np.max(np.abs(a - b))


def test_planted_mu_sign_is_caught():
    err = _free_field_error(lambda u, x: W.dw_apply(u, x, M_W, -0.3, g5=True))
    assert err > 1e-3


def test_planted_mass_is_caught():
    err = _free_field_error(lambda u, x: W.dw_apply(u, x, M_W + 0.1, 0.3, g5=True))
    assert err > 1e-3


def test_planted_transposed_link_is_caught():
    dims = (2, 4, 2, 4)
    u = latgen.random_gauge(dims, 0.9, 2)
    ut = np.swapaxes(u, -1, -2)  # U^T instead of U: same free field, wrong colour algebra
    x = latgen.random_sources(dims, 1, 3)[0]
    g = latgen.random_site_su3(dims, 9)
    gx = np.einsum("...ab,...sb->...sa", g, x)
    lhs = W.dw_apply(np.swapaxes(W.gauge_transform(u, g), -1, -2), gx, M_W, 0.0)
    rhs = np.einsum("...ab,...sb->...sa", g, W.dw_apply(ut, x, M_W, 0.0))
    assert np.max(np.abs(lhs - rhs)) > 1e-3
