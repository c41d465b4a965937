"""Exact matrix sign function, feasible only for small n.

Eq. (2) of the paper: for diagonalisable A = U diag(lambda_i) U^{-1},
f(A) = U diag(f(lambda_i)) U^{-1}; Sec. 1 fixes sgn(z) = sgn(Re z) for complex
eigenvalues.  ``sign_spectral`` is that definition written out with LAPACK's
eigensolvers (eigh for Hermitian input, eig plus a linear solve otherwise).

``sign_schur`` reaches the same matrix along a different route (a Schur form
ordered by the sign of Re(lambda) and a Sylvester solve); it does not use
eigenvectors and serves only to cross-check ``sign_spectral``.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _is_hermitian(a: np.ndarray, rtol: float = 1e-13) -> bool:
    return np.linalg.norm(a - a.conj().T) <= rtol * np.linalg.norm(a)


def sign_spectral(a: np.ndarray, hermitian: bool | None = None) -> np.ndarray:
    """sgn(A) = U diag(sgn Re lambda_i) U^{-1}  (Eq. (2) with sgn(z) = sgn(Re z))."""
    if hermitian is None:
        hermitian = _is_hermitian(a)
    if hermitian:
        w, q = np.linalg.eigh(a)
        return (q * np.sign(w)) @ q.conj().T
    w, r = np.linalg.eig(a)
    # U diag(s) U^{-1} = (U diag(s)) U^{-1}, with U^{-1} applied by a solve
    return np.linalg.solve(r.T, (r * np.sign(w.real)).T).T


def sign_schur(a: np.ndarray) -> np.ndarray:
    """sgn(A) from the Schur form with Re(lambda) > 0 ordered first.

    With A = Q T Q^dag and T = [[T11, T12], [0, T22]], sgn(T) = [[I, X], [0, -I]]
    where X solves T11 X - X T22 = 2 T12 (sgn(T) commutes with T).
    """
    t, q, k = sla.schur(a.astype(np.complex128), output="complex", sort="rhp")
    n = a.shape[0]
    s = np.zeros((n, n), dtype=np.complex128)
    s[:k, :k] = np.eye(k)
    s[k:, k:] = -np.eye(n - k)
    if 0 < k < n:
        s[:k, k:] = sla.solve_sylvester(t[:k, :k], -t[k:, k:], 2.0 * t[:k, k:])
    return q @ s @ q.conj().T


def sign_apply_exact(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sgn(A) x from the spectral definition."""
    return sign_spectral(a) @ x


def min_abs_re_eig(a: np.ndarray) -> float:
    """min |Re lambda| over the spectrum; the sign is undefined when it vanishes."""
    if _is_hermitian(a):
        return float(np.min(np.abs(np.linalg.eigvalsh(a))))
    return float(np.min(np.abs(np.linalg.eigvals(a).real)))
