"""Deflation of critical eigenvalues (Sec. 2, the paragraph after Eq. (4)).

Eigenvalues of A = gamma5 Dw(mu) close to the imaginary axis, where sgn jumps,
force a large Krylov space.  The paper takes m of them, lambda_i, with right
eigenvectors r_i (A r_i = lambda_i r_i) and left eigenvectors l_i
(l_i^dag A = lambda_i l_i^dag), normalised so that L_m^dag R_m = I, and splits

    f(A) x = R_m f(Lambda_m) (L_m^dag x) + f(A) (I - R_m L_m^dag) x.

The first term is exact.  The second is the Krylov approximation (non-nested
or nested) applied to the projected source, which has no component along the
deflated eigenvectors.  The paper assumes the eigenpairs are given (it cites
earlier work for computing them); ``critical_eigenpairs`` computes them for a
small dense A, which is all the tests need.  For Hermitian A (mu = 0) the left
and right eigenvectors coincide and are orthonormal.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import nested


def critical_eigenpairs(a: np.ndarray, m: int, hermitian: bool):
    """The m eigenvalues of dense A with the smallest |Re lambda|.

    Returns (lam, R, L): lam (m,) complex, R and L (n, m) with A R = R diag(lam),
    L^dag A = diag(lam) L^dag and L^dag R = I.
    """
    if hermitian:
        w, q = np.linalg.eigh(a)
        idx = np.argsort(np.abs(w), kind="stable")[:m]
        r = q[:, idx].astype(np.complex128)
        return w[idx].astype(np.complex128), r, r.copy()
    w, vl, vr = sla.eig(a, left=True, right=True)
    idx = np.argsort(np.abs(w.real), kind="stable")[:m]
    r = vr[:, idx]
    l = vl[:, idx]
    # biorthonormalise: with M = L^dag R, L M^{-dag} satisfies (L M^{-dag})^dag R = I
    mm = l.conj().T @ r
    l = l @ np.linalg.inv(mm).conj().T
    return w[idx], r, l


def sgn(lam: np.ndarray) -> np.ndarray:
    """sgn(z) = sgn(Re z) (Sec. 1); undefined on the imaginary axis."""
    re = np.asarray(lam).real
    if np.any(re == 0):
        raise ValueError("sgn is undefined for an eigenvalue on the imaginary axis")
    return np.sign(re)


def project(x: np.ndarray, r: np.ndarray, l: np.ndarray):
    """c = L^dag x and the projected source x - R c."""
    c = l.conj().T @ x
    return c, x - r @ c


def deflated_sign_apply(a_apply, a_dag_apply, x: np.ndarray, k: int, ell: int, hermitian: bool,
                        lam: np.ndarray, r: np.ndarray, l: np.ndarray, **kw):
    """sgn(A) x with the eigenpairs (lam, R, L) treated exactly.

    The Krylov part is ``nested.sign_apply`` (ell = 0: non-nested) on the
    projected source; a projected source that is exactly zero contributes
    nothing.  Returns (y, info) with y shaped like x.
    """
    xf = x.reshape(-1)
    m = len(lam)
    if m == 0:
        return nested.sign_apply(a_apply, a_dag_apply, x, k, ell, hermitian, **kw)
    c, xp = project(xf, r, l)
    y = r @ (sgn(lam) * c)
    info = {"c": c, "projected_norm": float(np.linalg.norm(xp))}
    if info["projected_norm"] > 0.0:
        yk, kinfo = nested.sign_apply(a_apply, a_dag_apply, xp.reshape(x.shape), k, ell, hermitian, **kw)
        y = y + yk.reshape(-1)
        info.update(kinfo)
    return y.reshape(x.shape), info
