"""A source on which two-sided Lanczos meets a serious breakdown at its first
step (Sec. 2: s = w_hat^dag v_hat vanishes while v_hat and w_hat do not).

In the free field a plane wave exp(i p.x) times a spinor s (colour 0) keeps
the recurrence in the four spinor directions at momentum p, where gamma5
Dw(mu) acts as the 4 x 4 matrix M = M(p).  With v_0 = w_0 = s / |s| the first
step gives s_1 = w_0^dag M^2 v_0 - (w_0^dag M v_0)^2, so a spinor with
(s^dag M^2 s)(s^dag s) = (s^dag M s)^2 that is not an eigenvector of M breaks
the recurrence down.  For mu != 0, M is not normal and such spinors exist;
they are found here by least squares from seeded starting points (the
search uses only the oracle's closed form of M).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares

from oracle import freefield as F

DIMS = (2, 2, 2, 4)
MOMENTUM = (0, 1, 0, 1)  # (nx, ny, nz, nt)


def momentum_matrix(m_w: float, mu: float, n=MOMENTUM) -> np.ndarray:
    nx, ny, nz, nt = n
    return F.g5dw_momentum(DIMS, m_w, mu)[nt, nz, ny, nx]


def breakdown_spinor(m_w: float, mu: float, seed: int = 1, trials: int = 20):
    """(s, r): unit spinor s and r = |w_hat^dag v_hat| / (|v_hat| |w_hat|) of the
    first two-sided Lanczos step on M from s, the smallest over the trials."""
    M = momentum_matrix(m_w, mu)

    def resid(z):
        s = z[:4] + 1j * z[4:]
        n = float(np.real(s.conj() @ s))
        val = (s.conj() @ M @ M @ s) * n - (s.conj() @ M @ s) ** 2
        return np.array([val.real, val.imag]) / n**2

    rng = np.random.default_rng(seed)
    best = (np.inf, None)
    for _ in range(trials):
        r = least_squares(resid, rng.standard_normal(8), xtol=1e-15, ftol=1e-15, gtol=1e-15)
        s = r.x[:4] + 1j * r.x[4:]
        s = s / np.linalg.norm(s)
        a = s.conj() @ M @ s
        vh = M @ s - a * s
        wh = M.conj().T @ s - np.conj(a) * s
        rr = abs(wh.conj() @ vh) / (np.linalg.norm(vh) * np.linalg.norm(wh))
        if rr < best[0]:
            best = (rr, s)
    return best[1], best[0]


def plane_wave(s: np.ndarray, n=MOMENTUM) -> np.ndarray:
    """exp(i p.x) s in colour 0, canonical layout (Lt, Lz, Ly, Lx, 4, 3)."""
    lx, ly, lz, lt = DIMS
    nx, ny, nz, nt = n
    px, py, pz, pt = F.momenta(DIMS)
    x = np.arange(lx)[None, None, None, :]
    y = np.arange(ly)[None, None, :, None]
    z = np.arange(lz)[None, :, None, None]
    t = np.arange(lt)[:, None, None, None]
    phase = np.exp(1j * (px[0, 0, 0, nx] * x + py[0, 0, ny, 0] * y + pz[0, nz, 0, 0] * z + pt[nt, 0, 0, 0] * t))
    psi = np.zeros((lt, lz, ly, lx, 4, 3), np.complex128)
    psi[..., :, 0] = phase[..., None] * s
    return psi
