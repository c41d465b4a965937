"""Krylov bases of Sec. 2: Hermitian Lanczos and two-sided Lanczos (2sL).

Both build a basis V_k of K_k(A, x) = span(x, Ax, ..., A^{k-1} x) starting
from v_1 = x / ||x|| and the tridiagonal Ritz matrix H_k of Eq. (3).

* Hermitian case (mu = 0): Lanczos gives orthonormal V_k with short
  recurrences and H_k = V_k^dag A V_k, real symmetric tridiagonal.
* Non-Hermitian case: 2sL builds V_k and W_k (bases of K_k(A, x) and
  K_k(A^dag, x)) with W_k^dag V_k = 1 and H_k = W_k^dag A V_k, again with short
  recurrences.  The paper does not fix how the normalisation is split between
  the two bases; this oracle takes w_1 = v_1 and, at each step,
  delta_{j+1} = sqrt(|s|), beta_{j+1} = s / delta_{j+1} with s = w_hat^dag v_hat,
  so that H_k has diagonal alpha, sub-diagonal delta and super-diagonal beta.
  The Ritz vector ||x|| V_k f(H_k) e_1 does not depend on that split.

No reorthogonalisation is done unless ``reorth`` is set (the paper keeps the
short recurrences; full re-(bi)orthogonalisation is used by the nested
method's inner level and by the exact-termination pin).

Test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Tridiag:
    """Tridiagonal Ritz matrix: diag ``alpha`` (k), sub ``delta`` (k-1), super ``beta`` (k-1)."""

    alpha: np.ndarray
    beta: np.ndarray
    delta: np.ndarray

    @property
    def k(self) -> int:
        return len(self.alpha)

    def dense(self) -> np.ndarray:
        k = self.k
        h = np.zeros((k, k), dtype=np.complex128)
        h[np.arange(k), np.arange(k)] = self.alpha
        if k > 1:
            h[np.arange(1, k), np.arange(k - 1)] = self.delta
            h[np.arange(k - 1), np.arange(1, k)] = self.beta
        return h

    def leading(self, m: int) -> "Tridiag":
        return Tridiag(self.alpha[:m].copy(), self.beta[: m - 1].copy(), self.delta[: m - 1].copy())


@dataclass
class KrylovResult:
    V: np.ndarray  # n x k, columns v_1 .. v_k
    H: Tridiag
    norm_x: float
    W: np.ndarray | None = None  # n x k for 2sL
    breakdown: int = 0  # step at which 2sL broke down (0 = none)


def lanczos(matvec, x: np.ndarray, k: int, reorth: bool = False) -> KrylovResult:
    """Hermitian Lanczos: w = A v_j - beta_{j-1} v_{j-1}; alpha_j = Re v_j^dag w;
    w -= alpha_j v_j; beta_j = ||w||; v_{j+1} = w / beta_j."""
    n = x.size
    nx = float(np.linalg.norm(x))
    V = np.zeros((n, k), dtype=np.complex128)
    alpha = np.zeros(k)
    beta = np.zeros(max(k - 1, 0))
    V[:, 0] = x.reshape(n) / nx
    bprev = 0.0
    for j in range(k):
        w = matvec(V[:, j])
        if j > 0:
            w = w - bprev * V[:, j - 1]
        alpha[j] = np.vdot(V[:, j], w).real
        w = w - alpha[j] * V[:, j]
        if reorth:
            for _ in range(2):
                w = w - V[:, : j + 1] @ (V[:, : j + 1].conj().T @ w)
        if j == k - 1:
            break
        bprev = float(np.linalg.norm(w))
        beta[j] = bprev
        V[:, j + 1] = w / bprev
    return KrylovResult(V=V, H=Tridiag(alpha.astype(np.complex128), beta.astype(np.complex128), beta.astype(np.complex128)), norm_x=nx)


def two_sided_lanczos(matvec, rmatvec, x: np.ndarray, k: int, reorth: bool = False,
                      breakdown_tol: float = 1e-14) -> KrylovResult:
    """Two-sided (biorthogonal) Lanczos with A = matvec, A^dag = rmatvec.

    alpha_j = w_j^dag A v_j
    v_hat   = A v_j - alpha_j v_j - beta_j v_{j-1}
    w_hat   = A^dag w_j - conj(alpha_j) w_j - delta_j w_{j-1}
    s = w_hat^dag v_hat, delta_{j+1} = sqrt|s|, beta_{j+1} = s / delta_{j+1}
    v_{j+1} = v_hat / delta_{j+1},  w_{j+1} = w_hat / conj(beta_{j+1}).
    A serious breakdown (|s| <= tol ||w_hat|| ||v_hat||) ends the basis early.
    """
    n = x.size
    nx = float(np.linalg.norm(x))
    V = np.zeros((n, k), dtype=np.complex128)
    W = np.zeros((n, k), dtype=np.complex128)
    alpha = np.zeros(k, dtype=np.complex128)
    beta = np.zeros(max(k - 1, 0), dtype=np.complex128)
    delta = np.zeros(max(k - 1, 0), dtype=np.complex128)
    V[:, 0] = x.reshape(n) / nx
    W[:, 0] = V[:, 0]
    brk = 0
    kk = k
    for j in range(k):
        av = matvec(V[:, j])
        aw = rmatvec(W[:, j])
        alpha[j] = np.vdot(W[:, j], av)
        vh = av - alpha[j] * V[:, j]
        wh = aw - np.conj(alpha[j]) * W[:, j]
        if j > 0:
            vh = vh - beta[j - 1] * V[:, j - 1]
            wh = wh - delta[j - 1] * W[:, j - 1]
        if reorth:
            for _ in range(2):
                vh = vh - V[:, : j + 1] @ (W[:, : j + 1].conj().T @ vh)
                wh = wh - W[:, : j + 1] @ (V[:, : j + 1].conj().T @ wh)
        if j == k - 1:
            break
        s = np.vdot(wh, vh)
        if abs(s) <= breakdown_tol * np.linalg.norm(wh) * np.linalg.norm(vh):
            brk = j + 1
            kk = j + 1
            break
        d = np.sqrt(abs(s))
        b = s / d
        delta[j] = d
        beta[j] = b
        V[:, j + 1] = vh / d
        W[:, j + 1] = wh / np.conj(b)
    H = Tridiag(alpha[:kk].copy(), beta[: kk - 1].copy(), delta[: kk - 1].copy())
    return KrylovResult(V=V[:, :kk], W=W[:, :kk], H=H, norm_x=nx, breakdown=brk)
