"""Pins for the Roberts-Higham iteration, Eq. (4).

For a real scalar z > 0, n steps of s <- (s + 1/s)/2 give exactly
coth(2^n artanh(min(z, 1/z))) (a closed form independent of the iteration);
on a diagonalisable matrix the iteration acts eigenvalue by eigenvalue; it
converges quadratically (Sec. 2) and its limit is the spectral sign.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import rh as R


@pytest.mark.parametrize("z", [0.01, 0.3, 0.999, 1.7, 42.0])
def test_scalar_closed_form(z):
    zz = min(z, 1.0 / z)
    for n in range(0, 8):
        exact = 1.0 / np.tanh(2.0**n * np.arctanh(zz))
        got = R.rh_scalar(z, n) if n > 0 else zz if z < 1 else exact
        if n > 0:
            assert abs(got - exact) <= 1e-13 * abs(exact)


def test_negative_scalar_is_odd():
    for n in range(1, 6):
        assert R.rh_scalar(-0.37, n) == pytest.approx(-R.rh_scalar(0.37, n), rel=1e-15)


def test_matrix_acts_eigenvaluewise():
    rng = np.random.default_rng(1)
    n = 12
    lam = np.concatenate([rng.uniform(0.05, 3.0, 6), -rng.uniform(0.05, 3.0, 6)])
    q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = q @ np.diag(lam) @ np.linalg.inv(q)
    s, it, _ = R.roberts_higham(a)
    assert np.linalg.norm(s - q @ np.diag(np.sign(lam)) @ np.linalg.inv(q)) < 1e-9 * np.linalg.norm(s)
    # four unscaled steps on the matrix equal four scalar steps per eigenvalue
    s4, _, _ = R.roberts_higham(a, tol=0.0, maxit=4)
    d4 = np.array([R.rh_scalar(l, 4) for l in lam])
    assert np.linalg.norm(s4 - q @ np.diag(d4) @ np.linalg.inv(q)) < 1e-9 * np.linalg.norm(s4)


def test_converges_to_spectral_sign_complex():
    rng = np.random.default_rng(2)
    n = 60
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a += 0.3 * np.diag(np.sign(rng.standard_normal(n)))
    s, it, change = R.roberts_higham(a)
    assert it < 40
    ref = D.sign_spectral(a, hermitian=False)
    assert np.linalg.norm(s - ref) < 1e-9 * np.linalg.norm(ref)


def test_quadratic_convergence():
    # error e_{n+1} ~ e_n^2 once in the asymptotic regime: on a scalar,
    # (s-1)/(s+1) squares at every step exactly.
    s = 5.0
    for _ in range(3):
        r0 = (s - 1) / (s + 1)
        s = 0.5 * (s + 1 / s)
        r1 = (s - 1) / (s + 1)
        assert r1 == pytest.approx(r0 * r0, rel=1e-9)


def test_scaling_keeps_limit():
    rng = np.random.default_rng(4)
    n = 30
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    s0, it0, _ = R.roberts_higham(a)
    s1, it1, _ = R.roberts_higham(a, scale=R.determinant_scale)
    assert np.linalg.norm(s0 - s1) < 1e-9 * np.linalg.norm(s0)
    assert it1 <= it0
