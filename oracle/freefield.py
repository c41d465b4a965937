"""Free field (all links U = 1): gamma5 Dw(mu) and its sign in momentum space.

For U = 1 the operator is diagonal in momentum.  A plane wave
psi(x) = exp(i p.x) chi, with p_j = 2 pi n_j / L_j in space and
p_t = (2 n_t + 1) pi / L_t in time (antiperiodic), satisfies
Dw(mu) psi = Dw(p) psi with

    Dw(p) = m_w + sum_nu (1 - cos q_nu) + i sum_nu gamma_nu sin q_nu,
    q_j = p_j,  q_t = p_t - i mu,

so the chemical potential of Sec. 1 shifts the temporal momentum into the
complex plane.  sgn(gamma5 Dw(mu)) then acts on each momentum through the
4 x 4 matrix sgn(gamma5 Dw(p)), obtained here from its eigen-decomposition
(Eq. (2)).  This gives an exact reference at any lattice volume.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .dense import sign_spectral
from .wilson import gamma5, gamma_matrices


def momenta(dims):
    """Arrays (px, py, pz, pt) broadcastable to (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    px = 2 * np.pi * np.arange(lx) / lx
    py = 2 * np.pi * np.arange(ly) / ly
    pz = 2 * np.pi * np.arange(lz) / lz
    pt = 2 * np.pi * np.arange(lt) / lt + np.pi / lt
    return (px[None, None, None, :], py[None, None, :, None], pz[None, :, None, None], pt[:, None, None, None])


def g5dw_momentum(dims, m_w: float, mu: float) -> np.ndarray:
    """gamma5 Dw(p) for every momentum, shape (Lt, Lz, Ly, Lx, 4, 4)."""
    g = gamma_matrices()
    g5 = gamma5()
    p = momenta(dims)
    q = [p[0] + 0j, p[1] + 0j, p[2] + 0j, p[3] - 1j * mu]
    shape = np.broadcast_shapes(*(qq.shape for qq in q))
    d = np.zeros(shape + (4, 4), dtype=np.complex128)
    scal = m_w + sum(1 - np.cos(qq) for qq in q)
    d += np.broadcast_to(scal, shape)[..., None, None] * np.eye(4)
    for nu in range(4):
        d += 1j * np.broadcast_to(np.sin(q[nu]), shape)[..., None, None] * g[nu]
    return np.einsum("st,...tu->...su", g5, d)


def _to_momentum(psi: np.ndarray) -> np.ndarray:
    lt = psi.shape[0]
    tw = np.exp(-1j * np.pi * np.arange(lt) / lt)[:, None, None, None, None, None]
    return np.fft.fftn(psi * tw, axes=(0, 1, 2, 3))


def _from_momentum(phi: np.ndarray) -> np.ndarray:
    lt = phi.shape[0]
    tw = np.exp(1j * np.pi * np.arange(lt) / lt)[:, None, None, None, None, None]
    return np.fft.ifftn(phi, axes=(0, 1, 2, 3)) * tw


def apply_momentum(psi: np.ndarray, mats: np.ndarray) -> np.ndarray:
    """Apply a per-momentum 4 x 4 spin matrix to psi (Lt, Lz, Ly, Lx, 4, 3)."""
    phi = _to_momentum(psi)
    phi = np.einsum("...st,...tc->...sc", mats, phi)
    return _from_momentum(phi)


def g5dw_apply_free(psi: np.ndarray, m_w: float, mu: float) -> np.ndarray:
    """gamma5 Dw(mu) psi for U = 1, through momentum space."""
    lt, lz, ly, lx = psi.shape[:4]
    return apply_momentum(psi, g5dw_momentum((lx, ly, lz, lt), m_w, mu))


def sign_matrices(dims, m_w: float, mu: float) -> np.ndarray:
    """sgn(gamma5 Dw(p)) for every momentum, shape (Lt, Lz, Ly, Lx, 4, 4)."""
    m = g5dw_momentum(dims, m_w, mu)
    flat = m.reshape(-1, 4, 4)
    out = np.empty_like(flat)
    herm = mu == 0.0
    for i in range(flat.shape[0]):
        out[i] = sign_spectral(flat[i], hermitian=herm)
    return out.reshape(m.shape)


def sign_apply_free(psi: np.ndarray, m_w: float, mu: float) -> np.ndarray:
    """sgn(gamma5 Dw(mu)) psi for U = 1, exact to rounding at any volume."""
    lt, lz, ly, lx = psi.shape[:4]
    return apply_momentum(psi, sign_matrices((lx, ly, lz, lt), m_w, mu))


def min_abs_re_eig(dims, m_w: float, mu: float) -> float:
    """Smallest |Re lambda| of gamma5 Dw(mu) at U = 1."""
    m = g5dw_momentum(dims, m_w, mu).reshape(-1, 4, 4)
    return float(np.min(np.abs(np.linalg.eigvals(m).real)))
