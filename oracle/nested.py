"""Non-nested and nested Krylov approximations of sgn(A) x.

Non-nested (Sec. 2, Eq. (3) with Eq. (4)):
    sgn(A) x ~ ||x|| V_k sgn(H_k) e_1,  sgn(H_k) by Roberts-Higham.

Nested (Sec. 3, Eq. (5) with the preconditioning step of Eq. (6)):
    sgn(H_k) e_1 = sgn(B) e_1 with B = H_k + H_k^{-1}, and
    sgn(B) e_1 ~ V_l sgn(H_l) e_1^{(l)} in the inner Krylov space K_l(B, e_1),
    so sgn(A) x ~ ||x|| V_k V_l sgn(H_l) e_1^{(l)}.

The paper names the inner approximation but not its basis construction.  This
oracle builds it with the same family as the outer level (Lanczos for
Hermitian H_k, two-sided Lanczos otherwise, both starting from e_1) with full
re-(bi)orthogonalisation, which costs O(k l^2) and keeps the small bases
well conditioned.  H_k^{-1} is applied through a dense LU solve.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .krylov import KrylovResult, Tridiag, lanczos, two_sided_lanczos
from .rh import roberts_higham


def outer_basis(a_apply, a_dag_apply, x: np.ndarray, k: int, hermitian: bool,
                reorth: bool = False) -> KrylovResult:
    """Outer basis of K_k(A, x): Lanczos at mu = 0, 2sL otherwise (Sec. 2)."""
    if hermitian:
        return lanczos(a_apply, x, k, reorth=reorth)
    return two_sided_lanczos(a_apply, a_dag_apply, x, k, reorth=reorth)


def rh_sign_e1(h: np.ndarray, **kw):
    """sgn(H) e_1 by the Roberts-Higham iteration; returns (vector, iterations)."""
    s, it, _ = roberts_higham(h, **kw)
    return s[:, 0].copy(), it


def inner_basis(b: np.ndarray, ell: int, hermitian: bool) -> KrylovResult:
    """Inner basis of K_l(B, e_1) with full re-(bi)orthogonalisation."""
    k = b.shape[0]
    e1 = np.zeros(k, dtype=np.complex128)
    e1[0] = 1.0
    if hermitian:
        return lanczos(lambda v: b @ v, e1, ell, reorth=True)
    bh = b.conj().T
    return two_sided_lanczos(lambda v: b @ v, lambda w: bh @ w, e1, ell, reorth=True)


def arnoldi(b: np.ndarray, ell: int, tol: float = 1e-14):
    """Arnoldi basis of K_l(B, e_1): V (k x m) with orthonormal columns and the
    m x m upper Hessenberg H = V^dag B V, from the recurrence
    h_{ji} = v_j^dag (B v_i) (j <= i), w = B v_i - sum_j h_{ji} v_j,
    h_{i+1,i} = ||w||, v_{i+1} = w / h_{i+1,i}, with the subtraction done twice
    (classical Gram-Schmidt with one reorthogonalisation) and the second
    pass's coefficients added to the first's.  Stops early (m < l) when the
    space becomes invariant (h_{i+1,i} <= tol ||B v_i||)."""
    k = b.shape[0]
    V = np.zeros((k, ell), np.complex128)
    H = np.zeros((ell, ell), np.complex128)
    V[0, 0] = 1.0
    for i in range(ell):
        w = b @ V[:, i]
        nw = np.linalg.norm(w)
        for _ in range(2):
            c = V[:, : i + 1].conj().T @ w
            w = w - V[:, : i + 1] @ c
            H[: i + 1, i] += c
        if i + 1 == ell:
            return V, H
        h = np.linalg.norm(w)
        if h <= tol * nw:
            return V[:, : i + 1], H[: i + 1, : i + 1]
        H[i + 1, i] = h
        V[:, i + 1] = w / h
    return V, H


def small_sign(H: Tridiag, ell: int, hermitian: bool, precondition: bool = True, inner: str = "same", **rhkw):
    """The k-vector z with sgn(A) x ~ ||x|| V_k z.

    ell == 0 selects the non-nested method, z = sgn(H_k) e_1.  Otherwise the
    nested method: z = V_l sgn(H_l) e_1^{(l)} with the inner space built on
    B = H_k + H_k^{-1} (``precondition``) or on H_k itself (the naive nesting
    of Sec. 3, kept only as a test pin), by the outer level's family
    (``inner = "same"``) or by Arnoldi (``"arnoldi"``).  Returns (z, info).
    """
    h = H.dense()
    k = h.shape[0]
    if ell == 0:
        z, it = rh_sign_e1(h, **rhkw)
        return z, {"rh_iters": it, "ell": 0}
    ell = min(ell, k)
    b = h + np.linalg.solve(h, np.eye(k)) if precondition else h
    if inner == "arnoldi":
        vl, hl = arnoldi(b, ell)
        y, it = rh_sign_e1(hl, **rhkw)
        return vl @ y, {"rh_iters": it, "ell": hl.shape[0], "H_ell": hl}
    ib = inner_basis(b, ell, hermitian)
    hl = ib.H.dense()
    y, it = rh_sign_e1(hl, **rhkw)
    z = ib.V[:, : hl.shape[0]] @ y
    return z, {"rh_iters": it, "ell": hl.shape[0], "H_ell": ib.H}


def sign_apply(a_apply, a_dag_apply, x: np.ndarray, k: int, ell: int, hermitian: bool,
               precondition: bool = True, inner: str = "same", **rhkw):
    """sgn(A) x by the non-nested (ell = 0) or nested (ell > 0) method.

    Returns (y, info) with y shaped like x.
    """
    kr = outer_basis(a_apply, a_dag_apply, x.reshape(-1), k, hermitian)
    z, info = small_sign(kr.H, ell, hermitian, precondition, inner, **rhkw)
    y = kr.norm_x * (kr.V @ z)
    info.update({"k": kr.H.k, "H": kr.H, "breakdown": kr.breakdown})
    return y.reshape(x.shape), info


def convergence_estimate(H: Tridiag, ell: int, hermitian: bool, d: int, inner: str = "same", **rhkw) -> float:
    """Relative change of the small-problem vector between k - d and k outer steps.

    est = ||z^{(k)} - [z^{(k-d)}; 0]|| / ||z^{(k)}||.  The paper defines no
    estimator.  With an orthonormal outer basis (Lanczos, mu = 0) it equals
    ||y_k - y_{k-d}|| / ||y_k|| and is pinned between the true errors against
    the exact sign; on the two-sided coefficients (mu != 0) it is a heuristic.
    """
    k = H.k
    z1, _ = small_sign(H, ell, hermitian, inner=inner, **rhkw)
    z0, _ = small_sign(H.leading(k - d), min(ell, k - d) if ell else 0, hermitian, inner=inner, **rhkw)
    diff = z1.copy()
    diff[: k - d] -= z0
    return float(np.linalg.norm(diff) / np.linalg.norm(z1))
