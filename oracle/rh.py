"""Roberts-Higham iteration for the matrix sign function, Eq. (4).

S_0 = A, S_{n+1} = (S_n + S_n^{-1}) / 2, which converges quadratically to
sgn(A) when A has no eigenvalue on the imaginary axis.  The paper gives no
stopping rule; this oracle stops when ||S_{n+1} - S_n||_F <= tol ||S_{n+1}||_F,
or when the change stops shrinking once it is already tiny (rounding floor),
or after ``maxit`` iterations.  The inverse is LAPACK's LU with partial
pivoting (numpy.linalg.inv).

``scale`` optionally multiplies S_n by a positive factor mu_n before the
update; sgn(mu S) = sgn(S) for mu > 0 (the scalar argument of Eq. (7) holds
for mu z as well), so scaling changes only the iteration count.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def roberts_higham(a: np.ndarray, tol: float = 1e-13, maxit: int = 100, scale=None):
    """Return (S, iterations, last relative change)."""
    s = np.array(a, dtype=np.complex128, copy=True)
    prev = np.inf
    it = 0
    change = np.inf
    for it in range(1, maxit + 1):
        if scale is not None:
            m = scale(it - 1, s)
            if m is not None:
                s = m * s
        s_new = 0.5 * (s + np.linalg.inv(s))
        change = np.linalg.norm(s_new - s) / np.linalg.norm(s_new)
        s = s_new
        if change <= tol:
            break
        if change < 1e-6 and change > 0.5 * prev:
            break  # stagnated at the rounding floor
        prev = change
    return s, it, change


def determinant_scale(it: int, s: np.ndarray):
    """Determinant scaling mu = |det S|^{-1/n} (an option; not the paper's iteration)."""
    sign, logdet = np.linalg.slogdet(s)
    return float(np.exp(-logdet.real / s.shape[0]))


def rh_scalar(z: float, n: int) -> float:
    """n unscaled RH steps on a real scalar z: s <- (s + 1/s) / 2."""
    s = z
    for _ in range(n):
        s = 0.5 * (s + 1.0 / s)
    return s
