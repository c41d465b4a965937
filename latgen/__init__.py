"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module produces gauge fields and source vectors only.  It contains none
of the arithmetic of the sign-function method (no Dirac operator, no Krylov
step, no matrix sign), so both sides of a parity test can draw the same
inputs from it without sharing any of the code under test.

Conventions (the paper fixes none of them; Sec. 1 only names the
Wilson-Dirac operator with the Hasenfratz-Karsch chemical potential):

* lattice dims are ``(Lx, Ly, Lz, Lt)``; arrays are indexed
  ``[t, z, y, x, ...]`` so that x runs fastest in memory, and the site index
  is ``((t*Lz + z)*Ly + y)*Lx + x``;
* a gauge field has shape ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` complex128, where
  ``U[..., nu, a, b]`` is the SU(3) link from site x to x + nu-hat
  (nu = 0, 1, 2, 3 for x, y, z, t);
* a spinor field has shape ``(Lt, Lz, Ly, Lx, 4, 3)`` complex128
  (spin, colour), i.e. vector index ``site*12 + spin*3 + colour``.

Gauge links are ``U = exp(i*eps*M)`` with ``M = sum_a c_a lambda_a / 2``,
``c_a ~ N(0, 1)`` and lambda_a the Gell-Mann matrices, then re-unitarised to
SU(3).  The width ``eps`` sets how rough the field is and therefore how many
eigenvalues of gamma5*Dw lie close to the imaginary axis; it stands in for
the thermalised configurations of the paper, which are not available.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "random_gauge",
    "unit_gauge",
    "random_sources",
    "random_site_su3",
    "uneven_ell",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Project (..., 3, 3) matrices onto SU(3) row by row.

    Row 0 is normalised, row 1 is made orthogonal to row 0 and normalised,
    and row 2 is the complex conjugate of the cross product of rows 0 and 1,
    which makes the determinant exactly one.
    """
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _su3_from_coeffs(c: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*sum_a c_a lambda_a/2) for coefficient arrays of shape (..., 8)."""
    lam = gell_mann()
    m = np.einsum("...a,aij->...ij", c, lam) * 0.5
    w, q = np.linalg.eigh(m)
    ph = np.exp(1j * eps * w)
    u = np.einsum("...ij,...j,...kj->...ik", q, ph, np.conj(q))
    return _reunitarise(u)


def random_gauge(dims, eps: float, seed: int = 0) -> np.ndarray:
    """Seeded random SU(3) gauge field near the identity.

    ``dims = (Lx, Ly, Lz, Lt)``; returns complex128 of shape
    ``(Lt, Lz, Ly, Lx, 4, 3, 3)``.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((lt, lz, ly, lx, 4, 8))
    return _su3_from_coeffs(c, eps)


def unit_gauge(dims) -> np.ndarray:
    """The free field U = 1 on every link."""
    lx, ly, lz, lt = (int(d) for d in dims)
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_site_su3(dims, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site (a gauge transformation), shape (Lt,Lz,Ly,Lx,3,3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng([seed, 7])
    c = rng.standard_normal((lt, lz, ly, lx, 8))
    return _su3_from_coeffs(c, 2.0)


def random_sources(dims, nsrc: int = 1, seed: int = 0) -> np.ndarray:
    """Complex Gaussian sources, shape (nsrc, Lt, Lz, Ly, Lx, 4, 3) complex128."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng([seed, 1])
    r = rng.standard_normal((nsrc, lt, lz, ly, lx, 4, 3, 2))
    return r[..., 0] + 1j * r[..., 1]


def uneven_ell(nsrc: int = 32, lo: int = 40, hi: int = 300, seed: int = 0) -> np.ndarray:
    """Per-source inner Krylov sizes drawn uniformly from [lo, hi]."""
    rng = np.random.default_rng([seed, 2])
    return rng.integers(lo, hi + 1, nsrc)


def mlp_init(seed: int = 0, nin: int = 16, nh: int = 64, nout: int = 4) -> np.ndarray:
    """Seeded initial parameters of a nin-nh-nh-nh-nout network, flat float32 in
    the order W1, b1, W2, b2, W3, b3, W4, b4 followed by the feature
    standardisation (mean = 0, inverse std = 1).  Hidden weights are uniform
    with the Glorot bound sqrt(6 / (fan_in + fan_out)); the output layer and
    all biases start at zero (the untrained network outputs 0).  Random
    numbers only, no arithmetic of the method."""
    rng = np.random.default_rng([seed, 7])
    parts = []
    for fi, fo, gain in ((nin, nh, 1.0), (nh, nh, 1.0), (nh, nh, 1.0), (nh, nout, 0.0)):
        bound = gain * np.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-bound, bound, size=fo * fi))
        parts.append(np.zeros(fo))
    parts.append(np.zeros(nin))
    parts.append(np.ones(nin))
    return np.concatenate(parts).astype(np.float32)
