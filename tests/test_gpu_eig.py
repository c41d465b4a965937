"""GPU parity of the Hermitian critical-eigenpair solver (deflation, Sec. 2, mu = 0).

* 2x2x4x4: the 16 eigenvalues of gamma5 Dw(0) smallest in modulus against the
  oracle's dense eigen-decomposition (1e-10), orthonormal eigenvectors, and
  residuals |H r - lambda r| recomputed with the oracle's stencil;
* 2x2x4x4 free field: an exactly symmetric cluster lambda = +1, -1 (24 each)
  against the closed-form momentum-space spectrum;
* what they are for: deflating a nested sign application on 2x4x4x4 with the
  GPU's own eigenpairs is as accurate as with the dense ones, and more
  accurate than no deflation at the same k;
* invalid arguments.
"""
import numpy as np
import pytest

import latgen
from oracle import deflation as DF
from oracle import dense as D
from oracle import freefield as FF
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, make_lattice, nk, rel, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _eig(lat, dims, m, p, degree=20, tol=1e-11, maxit=80, seed=11):
    b = nk()
    V0 = to_dev(latgen.random_sources(dims, p, seed))
    R = torch_cuda().empty(m * V0.numel() // p, dtype=V0.dtype, device=V0.device)
    lam, passes, resid, rc = b.nk_eig_hermitian_device(lat.h, M_W, m, p, degree, tol, maxit, V0, R)
    return lam, to_host(R).reshape(m, -1).T, passes, resid, rc


def test_matches_dense():
    dims = (2, 2, 4, 4)
    banner("eigensolver 2x2x4x4 mu=0 m=16 p=24")
    lat, u = make_lattice(dims, 0.8, seed=0)
    lam, r, passes, resid, rc = _eig(lat, dims, 16, 24)
    print(f"passes {passes} resid {resid:.2e}", flush=True)
    assert rc == 0 and resid <= 1e-11 * 11.0
    lam_d, _, _ = DF.critical_eigenpairs(W.dense_matrix(u, M_W, 0.0), 16, True)
    assert np.max(np.abs(lam - lam_d.real)) < 1e-10
    assert np.linalg.norm(r.conj().T @ r - np.eye(16)) < 1e-12
    shape = (4, 4, 2, 2, 4, 3)
    for i in range(16):
        hr = W.a_apply(u, r[:, i].reshape(shape), M_W, 0.0).reshape(-1)
        assert np.linalg.norm(hr - lam[i] * r[:, i]) < 2e-10
    lat.close()


@pytest.mark.parametrize("m", [48, 40])
def test_free_field_symmetric_pairs(m):
    """U = 1 on 2x2x4x4 at m_w = -1: the smallest |lambda| of gamma5 Dw(0) is
    1, with 24 eigenvectors at +1 and 24 at -1 (the plane waves of the lowest
    temporal momenta and their doublers), an exactly symmetric cluster that
    H^2 cannot split.  Against the closed-form momentum-space spectrum: at
    m = 48 the sorted eigenvalues, at m = 40 (inside the cluster) |lambda| = 1;
    both with residuals from the oracle's free-field operator and orthonormal
    vectors."""
    dims = (2, 2, 4, 4)
    banner(f"eigensolver free field 2x2x4x4 mu=0 m={m} p=64")
    lat, u = make_lattice(dims, 0.0, unit=True)
    lam, r, passes, resid, rc = _eig(lat, dims, m, 64, degree=20, tol=1e-11, maxit=60)
    print(f"passes {passes} resid {resid:.2e}", flush=True)
    assert rc == 0 and resid <= 1e-11 * 11.0
    ev = np.repeat(np.linalg.eigvals(FF.g5dw_momentum(dims, M_W, 0.0).reshape(-1, 4, 4)).ravel().real, 3)
    exact = np.sort(ev[np.argsort(np.abs(ev), kind="stable")[:48]])
    assert np.max(np.abs(exact)) - 1.0 < 1e-12 and np.sum(exact > 0) == 24
    if m == 48:
        assert np.max(np.abs(np.sort(lam) - exact)) < 1e-10
    else:
        assert np.max(np.abs(np.abs(lam) - 1.0)) < 1e-10
    assert np.linalg.norm(r.conj().T @ r - np.eye(m)) < 1e-12
    shape = (4, 4, 2, 2, 4, 3)
    for i in range(m):
        hr = FF.g5dw_apply_free(r[:, i].reshape(shape), M_W, 0.0).reshape(-1)
        assert np.linalg.norm(hr - lam[i] * r[:, i]) < 2e-10
    lat.close()


def test_deflation_with_gpu_eigenpairs():
    dims = (2, 4, 4, 4)
    banner("eigensolver 2x4x4x4 mu=0: deflation with the GPU's eigenpairs")
    lat, u = make_lattice(dims, 0.8, seed=0)
    lam, r, passes, resid, rc = _eig(lat, dims, 16, 24)
    assert rc == 0
    a = W.dense_matrix(u, M_W, 0.0)
    x = latgen.random_sources(dims, 1, 0)[0]
    exact = D.sign_spectral(a, hermitian=True) @ x.reshape(-1)
    b = nk()
    p = b.nk_sign_params_default(mu=0.0, m_w=M_W, k=200, ell=50)
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    R = to_dev(r.T)
    b.nk_sign_apply_deflated_device(lat.h, p, lam.astype(np.complex128), R, R, dx, dy)
    e_gpu = rel(to_host(dy), exact)
    lam_d, r_d, l_d = DF.critical_eigenpairs(a, 16, True)
    b.nk_sign_apply_deflated_device(lat.h, p, lam_d, to_dev(r_d.T), to_dev(l_d.T), dx, dy)
    e_dense = rel(to_host(dy), exact)
    b.nk_sign_apply_device(lat.h, p, dx, dy)
    e_none = rel(to_host(dy), exact)
    print(f"k=200: deflated (GPU eigenpairs) {e_gpu:.2e}, (dense) {e_dense:.2e}, none {e_none:.2e}", flush=True)
    assert e_gpu < 1.5 * e_dense + 1e-12
    assert e_gpu < e_none / 4
    lat.close()


def test_invalid_arguments():
    dims = (2, 2, 2, 2)
    lat, u = make_lattice(dims, 0.8, seed=0)
    b = nk()
    V0 = to_dev(latgen.random_sources(dims, 8, 1))
    R = torch_cuda().empty(4 * 192, dtype=V0.dtype, device=V0.device)
    for m, p, deg, tol, it in ((0, 8, 10, 1e-8, 5), (9, 8, 10, 1e-8, 5), (4, 8, 0, 1e-8, 5), (4, 8, 10, 0.0, 5),
                               (4, 8, 10, 1e-8, 0), (4, 129, 10, 1e-8, 5)):
        with pytest.raises(b.NKError) as ei:
            b.nk_eig_hermitian_device(lat.h, M_W, m, p, deg, tol, it, V0, R)
        assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_eig_hermitian_device(lat.h, M_W, 4, 8, 10, 1e-8, 5, V0, V0[: 4 * 192])
    assert ei.value.code == b.NK_EINVAL
    lat.close()


def test_full_size():
    """16^4 (the benchmark lattice at mu = 0): converged residuals, checked
    again with the library's own stencil call, and orthonormal vectors."""
    dims = (16, 16, 16, 16)
    banner("eigensolver 16^4 mu=0 m=16 p=32 degree=40")
    lat, u = make_lattice(dims, 0.8, seed=0)
    lam, r, passes, resid, rc = _eig(lat, dims, 16, 32, degree=40, tol=1e-10, maxit=100)
    print(f"passes {passes} resid {resid:.2e} |lam| {np.abs(lam).min():.4f}..{np.abs(lam).max():.4f}", flush=True)
    assert rc == 0 and resid <= 1.1e-9
    assert np.all(np.diff(np.abs(lam)) > -1e-9)
    assert np.linalg.norm(r.conj().T @ r - np.eye(16)) < 1e-11
    b = nk()
    for i in (0, 15):
        dr = to_dev(r[:, i])
        dh = torch_cuda().empty_like(dr)
        b.nk_apply_dw_device(lat.h, M_W, 0.0, True, dr, dh)
        assert np.linalg.norm(to_host(dh) - lam[i] * r[:, i]) < 1.2e-9
    lat.close()


def _eig_critical(lat, dims, mu, m, p, degree=20, tol=1e-11, maxit=120, seed=11):
    b = nk()
    V0 = to_dev(latgen.random_sources(dims, p, seed))
    nm = m * V0.numel() // p
    R = torch_cuda().empty(nm, dtype=V0.dtype, device=V0.device)
    L = torch_cuda().empty(nm, dtype=V0.dtype, device=V0.device)
    lam, passes, resid, rc = b.nk_eig_critical_device(lat.h, M_W, mu, m, p, degree, tol, maxit, V0, R, L)
    return lam, to_host(R).reshape(m, -1).T, to_host(L).reshape(m, -1).T, passes, resid, rc


@pytest.mark.parametrize("mu", [0.3, 0.0])
def test_critical_matches_dense(mu):
    """The two-sided solver (any mu) on 2x2x4x4, link width 0.8: the 16
    eigenvalues of gamma5 Dw(mu) nearest the imaginary axis against the
    oracle's dense eigen-decomposition (1e-10), A R = R Lambda and
    L^dag A = Lambda L^dag recomputed with the oracle's stencil (2e-10), and
    L^dag R = I (1e-10)."""
    dims = (2, 2, 4, 4)
    banner(f"critical eigensolver 2x2x4x4 mu={mu} m=16 p=24")
    lat, u = make_lattice(dims, 0.8, seed=0)
    lam, r, l, passes, resid, rc = _eig_critical(lat, dims, mu, 16, 24)
    print(f"[eig] mu={mu}: passes {passes} resid {resid:.2e}", flush=True)
    assert rc == 0
    lam_d, _, _ = DF.critical_eigenpairs(W.dense_matrix(u, M_W, mu), 16, mu == 0.0)
    # the same set (an eigenvalue's partner of equal |Re| may come in either order)
    for z in lam:
        assert np.min(np.abs(lam_d - z)) < 1e-10, z
    assert np.allclose(np.sort(np.abs(lam.real)), np.sort(np.abs(lam_d.real)), atol=1e-10)
    assert np.linalg.norm(l.conj().T @ r - np.eye(16)) < 1e-10
    shape = (4, 4, 2, 2, 4, 3)
    for i in range(16):
        ar = W.a_apply(u, r[:, i].reshape(shape), M_W, mu).reshape(-1)
        assert np.linalg.norm(ar - lam[i] * r[:, i]) < 2e-10 * np.linalg.norm(r[:, i])
        adl = W.a_apply(u, l[:, i].reshape(shape), M_W, -mu).reshape(-1)  # A^dag l = conj(lambda) l
        assert np.linalg.norm(adl - np.conj(lam[i]) * l[:, i]) < 2e-10 * np.linalg.norm(l[:, i])
    lat.close()


def test_deflation_with_gpu_critical_eigenpairs_mu03():
    """What they are for at mu = 0.3: deflating a nested sign application on
    2x4x4x4 with the GPU's own left and right eigenpairs is as accurate as
    with the dense ones, and more accurate than no deflation at the same k."""
    dims = (2, 4, 4, 4)
    mu = 0.3
    banner("critical eigensolver 2x4x4x4 mu=0.3: deflation with the GPU's eigenpairs")
    lat, u = make_lattice(dims, 0.8, seed=0)
    lam, r, l, passes, resid, rc = _eig_critical(lat, dims, mu, 16, 24)
    assert rc == 0
    a = W.dense_matrix(u, M_W, mu)
    x = latgen.random_sources(dims, 1, 0)[0]
    exact = D.sign_spectral(a, hermitian=False) @ x.reshape(-1)
    lam_d, r_d, l_d = DF.critical_eigenpairs(a, 16, False)
    b = nk()
    p = b.nk_sign_params_default(mu=mu, m_w=M_W, k=200, ell=50)
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    b.nk_sign_apply_deflated_device(lat.h, p, lam, to_dev(r.T), to_dev(l.T), dx, dy)
    e_gpu = rel(to_host(dy), exact)
    b.nk_sign_apply_deflated_device(lat.h, p, lam_d, to_dev(r_d.T), to_dev(l_d.T), dx, dy)
    e_dense = rel(to_host(dy), exact)
    b.nk_sign_apply_device(lat.h, p, dx, dy)
    e_none = rel(to_host(dy), exact)
    print(f"[eig] 2x4x4x4 mu=0.3 k=200 l=50: deflated (GPU pairs) {e_gpu:.2e}, (dense pairs) {e_dense:.2e}, "
          f"undeflated {e_none:.2e}", flush=True)
    assert e_gpu < 2.0 * e_dense + 1e-12
    assert e_gpu < 0.5 * e_none
    lat.close()


def test_critical_rejects_bad_arguments():
    b = nk()
    dims = (2, 2, 2, 2)
    lat, _ = make_lattice(dims, 0.5, seed=0)
    V0 = to_dev(latgen.random_sources(dims, 4, 1))
    R = torch_cuda().empty(2 * 192, dtype=V0.dtype, device=V0.device)
    L = torch_cuda().empty(2 * 192, dtype=V0.dtype, device=V0.device)
    with pytest.raises(b.NKError):
        b.nk_eig_critical_device(lat.h, M_W, 0.3, 5, 4, 10, 1e-10, 10, V0, R, L)  # m > p
    with pytest.raises(b.NKError):
        b.nk_eig_critical_device(lat.h, M_W, 0.3, 2, 4, 10, 1e-10, 10, V0, R, R)  # R and L overlap
    lat.close()
