"""The overlap operator and a linear solver on it (Sec. 1, Eq. (1)).

Dov(mu) = 1 + gamma5 sgn(gamma5 Dw(mu)).  With A = gamma5 Dw(mu) and
S = sgn(A), the adjoint is Dov^dag = 1 + S^dag gamma5, and S^dag = sgn(A^dag)
because A^dag has the conjugate eigenvalues (same real parts) with the
inverse-adjoint eigenvectors.  In this convention A^dag = gamma5 Dw(-mu), so
Dov(mu)^dag v = v + sgn(gamma5 Dw(-mu)) gamma5 v.

The paper motivates the sign computation by iterative solvers on Dov without
fixing one.  ``cgnr`` is the textbook conjugate-gradient method on the normal
equations Dov^dag Dov y = Dov^dag b (it minimises |b - Dov y| over growing
Krylov spaces), which needs Dov and Dov^dag only.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

G5 = np.array([1.0, 1.0, -1.0, -1.0])


def gamma5(v: np.ndarray) -> np.ndarray:
    """gamma5 = diag(1, 1, -1, -1) on the spin index of canonical (..., 4, 3) vectors."""
    shape = v.shape
    w = v.reshape(-1, 4, 3) * G5[None, :, None]
    return w.reshape(shape)


def dov_apply(sign_apply, x: np.ndarray) -> np.ndarray:
    """Dov x = x + gamma5 sgn(A) x, with sign_apply(v) = sgn(A) v."""
    return x + gamma5(sign_apply(x))


def dov_dag_apply(sign_dag_apply, x: np.ndarray) -> np.ndarray:
    """Dov^dag x = x + sgn(A^dag) gamma5 x, with sign_dag_apply(v) = sgn(A^dag) v."""
    return x + sign_dag_apply(gamma5(x))


def dense_dov(sign_matrix: np.ndarray) -> np.ndarray:
    """Dov as a dense matrix from the dense sgn(A) (canonical ordering)."""
    n = sign_matrix.shape[0]
    g = np.tile(np.repeat(G5, 3), n // 12)
    return np.eye(n) + g[:, None] * sign_matrix


def cgnr(dov, dov_dag, b: np.ndarray, tol: float, maxit: int):
    """Solve Dov y = b by CG on the normal equations, from y = 0.

    Stops when the recursively updated residual |r| <= tol |b|.  Returns
    (y, iterations, |r| / |b|, history of |r| / |b|).
    """
    bf = b.reshape(-1)
    y = np.zeros_like(bf)
    r = bf.copy()
    z = dov_dag(r)
    p = z.copy()
    zz = np.vdot(z, z).real
    nb = np.linalg.norm(bf)
    hist = [1.0]
    it = 0
    while it < maxit and hist[-1] > tol:
        it += 1
        w = dov(p)
        alpha = zz / np.vdot(w, w).real
        y = y + alpha * p
        r = r - alpha * w
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            break
        z = dov_dag(r)
        zz_new = np.vdot(z, z).real
        p = z + (zz_new / zz) * p
        zz = zz_new
    return y.reshape(b.shape), it, hist[-1], hist
