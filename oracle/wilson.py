"""Wilson-Dirac operator Dw(mu) and A = gamma5 Dw(mu), plain FP64.

Sec. 1 of the paper defines the overlap operator through sgn(gamma5 Dw(mu)),
Eq. (1), with Wilson mass -2 < m_w < 0 and the chemical potential entering
Dw as prescribed by Hasenfratz and Karsch.  The paper does not write Dw out;
this oracle fixes the standard form

  (Dw psi)(x) = (4 + m_w) psi(x)
      - 1/2 sum_nu [ e^{+mu d_{nu,t}} (1 - gamma_nu) U_nu(x) psi(x + nu)
                   + e^{-mu d_{nu,t}} (1 + gamma_nu) U_nu(x - nu)^dag psi(x - nu) ]

with periodic boundaries in x, y, z and antiperiodic ones in t (a hop that
wraps in t picks up a factor -1), chiral Euclidean gamma matrices and
gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1).  At mu = 0,
gamma5 Dw is Hermitian (Sec. 1).  Array conventions are those of ``latgen``.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

_SIGMA = np.array(
    [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128
)


def gamma_matrices() -> np.ndarray:
    """gamma_1..gamma_4 (index 0..3 = x, y, z, t) in the chiral basis, shape (4, 4, 4)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k][:2, 2:] = -1j * _SIGMA[k]
        g[k][2:, :2] = 1j * _SIGMA[k]
    g[3][:2, 2:] = np.eye(2)
    g[3][2:, :2] = np.eye(2)
    return g


def gamma5() -> np.ndarray:
    g = gamma_matrices()
    return g[0] @ g[1] @ g[2] @ g[3]


# lattice axis of direction nu in arrays indexed [t, z, y, x]
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def dims_of(psi: np.ndarray):
    """(Lx, Ly, Lz, Lt) of a spinor field of shape (Lt, Lz, Ly, Lx, 4, 3)."""
    lt, lz, ly, lx = psi.shape[:4]
    return (lx, ly, lz, lt)


def dw_apply(u: np.ndarray, psi: np.ndarray, m_w: float, mu: float, g5: bool = False) -> np.ndarray:
    """Dw(mu) psi (or gamma5 Dw(mu) psi when ``g5``), vectorised with np.roll.

    u: (Lt, Lz, Ly, Lx, 4, 3, 3); psi: (Lt, Lz, Ly, Lx, 4, 3).
    """
    g = gamma_matrices()
    one = np.eye(4)
    out = (4.0 + m_w) * psi
    for nu in range(4):
        ax = _AXIS[nu]
        unu = u[..., nu, :, :]
        # forward hop: U_nu(x) psi(x + nu)
        fwd = np.roll(psi, -1, axis=ax)
        # backward hop: U_nu(x - nu)^dag psi(x - nu)
        bwd = np.roll(psi, 1, axis=ax)
        ub = np.conj(np.swapaxes(np.roll(unu, 1, axis=ax), -1, -2))
        if nu == 3:
            fwd = fwd.copy()
            bwd = bwd.copy()
            fwd[-1] *= -1.0  # x + t wraps from t = Lt-1 to t = 0
            bwd[0] *= -1.0  # x - t wraps from t = 0 to t = Lt-1
        ef = np.exp(mu) if nu == 3 else 1.0
        eb = np.exp(-mu) if nu == 3 else 1.0
        uf = np.einsum("...ab,...sb->...sa", unu, fwd)
        ubp = np.einsum("...ab,...sb->...sa", ub, bwd)
        out = out - 0.5 * ef * np.einsum("st,...ta->...sa", one - g[nu], uf)
        out = out - 0.5 * eb * np.einsum("st,...ta->...sa", one + g[nu], ubp)
    if g5:
        out = np.einsum("st,...ta->...sa", gamma5(), out)
    return out


def dw_apply_loops(u: np.ndarray, psi: np.ndarray, m_w: float, mu: float, g5: bool = False) -> np.ndarray:
    """Same operator written as an explicit loop over sites and directions.

    Pure Python; only for tiny lattices (it cross-checks ``dw_apply``).
    """
    g = gamma_matrices()
    g5m = gamma5()
    lt, lz, ly, lx = psi.shape[:4]
    L = (lx, ly, lz, lt)
    out = np.zeros_like(psi)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    acc = (4.0 + m_w) * psi[t, z, y, x]
                    for nu in range(4):
                        f = list(c)
                        f[nu] += 1
                        sf = 1.0
                        if f[nu] == L[nu]:
                            f[nu] = 0
                            sf = -1.0 if nu == 3 else 1.0
                        b = list(c)
                        b[nu] -= 1
                        sb = 1.0
                        if b[nu] < 0:
                            b[nu] = L[nu] - 1
                            sb = -1.0 if nu == 3 else 1.0
                        ef = np.exp(mu) if nu == 3 else 1.0
                        eb = np.exp(-mu) if nu == 3 else 1.0
                        pf = psi[f[3], f[2], f[1], f[0]]
                        pb = psi[b[3], b[2], b[1], b[0]]
                        uf = u[t, z, y, x, nu]
                        ubk = u[b[3], b[2], b[1], b[0], nu]
                        hf = (uf @ pf.T).T  # colour rotation, spin untouched
                        hb = (np.conj(ubk).T @ pb.T).T
                        acc = acc - 0.5 * ef * sf * ((np.eye(4) - g[nu]) @ hf)
                        acc = acc - 0.5 * eb * sb * ((np.eye(4) + g[nu]) @ hb)
                    out[t, z, y, x] = g5m @ acc if g5 else acc
    return out


def a_apply(u, psi, m_w, mu):
    """A psi with A = gamma5 Dw(mu)."""
    return dw_apply(u, psi, m_w, mu, g5=True)


def a_dag_apply(u, psi, m_w, mu):
    """A^dag psi computed as the adjoint of the sum of hops, term by term.

    Written without using gamma5-hermiticity, so that the identity
    A(mu)^dag = A(-mu) can be tested against it: A^dag = Dw^dag gamma5.
    """
    g = gamma_matrices()
    one = np.eye(4)
    phi = np.einsum("st,...ta->...sa", gamma5(), psi)
    out = (4.0 + m_w) * phi
    for nu in range(4):
        ax = _AXIS[nu]
        unu = u[..., nu, :, :]
        ef = np.exp(mu) if nu == 3 else 1.0
        eb = np.exp(-mu) if nu == 3 else 1.0
        # adjoint of the forward hop x <- x+nu: maps phi(x) to site x+nu with
        # (1 - gamma)^dag U^dag; i.e. at site y it reads phi(y - nu).
        pb = np.roll(phi, 1, axis=ax)
        ub = np.conj(np.swapaxes(np.roll(unu, 1, axis=ax), -1, -2))
        if nu == 3:
            pb = pb.copy()
            pb[0] *= -1.0
        term = np.einsum("...ab,...sb->...sa", ub, pb)
        out = out - 0.5 * ef * np.einsum("st,...ta->...sa", (one - g[nu]).conj().T, term)
        # adjoint of the backward hop x <- x-nu: at site y it reads phi(y + nu)
        pf = np.roll(phi, -1, axis=ax)
        if nu == 3:
            pf = pf.copy()
            pf[-1] *= -1.0
        term = np.einsum("...ab,...sb->...sa", unu, pf)
        out = out - 0.5 * eb * np.einsum("st,...ta->...sa", (one + g[nu]).conj().T, term)
    return out


def dense_matrix(u, m_w, mu, g5=True) -> np.ndarray:
    """The n x n matrix of gamma5 Dw(mu) (or Dw(mu)), n = 12 V, by unit-vector application."""
    shape = u.shape[:4] + (4, 3)
    n = int(np.prod(shape))
    m = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        e[i] = 1.0
        m[:, i] = dw_apply(u, e.reshape(shape), m_w, mu, g5).reshape(n)
        e[i] = 0.0
    return m


def gauge_transform(u: np.ndarray, gsite: np.ndarray) -> np.ndarray:
    """U_nu(x) -> G(x) U_nu(x) G(x + nu)^dag, boundaries as for the lattice (links are periodic)."""
    out = np.empty_like(u)
    for nu in range(4):
        ax = _AXIS[nu]
        gf = np.roll(gsite, -1, axis=ax)
        out[..., nu, :, :] = gsite @ u[..., nu, :, :] @ np.conj(np.swapaxes(gf, -1, -2))
    return out
