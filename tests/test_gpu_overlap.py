"""GPU parity of the overlap operator (Eq. (1)) and the CGNR solver on it.

* Dov and Dov^dag on a 2x2x4x4 lattice against the dense Dov built from the
  exact sign (Schur route), at a k where the sign's Krylov error is below
  1e-12 (4e-13 at mu = 0.3 in the oracle): <= 1e-9;
* at 16^4 (the benchmark lattice, k = 500, l = 60): the adjoint identity
  <u, Dov v> = <Dov^dag u, v> and Ginsparg-Wilson, to the sign's accuracy;
* CGNR against np.linalg.solve on the dense Dov (2x2x4x4), and at 16^4 a
  solve whose true residual is checked with an independent application;
* edge cases: b = 0, an iteration cap, invalid arguments.
"""
import numpy as np
import pytest

import latgen
from oracle import dense as D
from oracle import overlap as O
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, make_lattice, nk, rel, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _params(**kw):
    return nk().nk_sign_params_default(m_w=M_W, **kw)


def _apply(lat, x, dagger, **kw):
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    info, rc = nk().nk_overlap_apply_device(lat.h, _params(**kw), dagger, dx, dy)
    return to_host(dy), rc


def _cdot(a, b):
    return complex(np.vdot(np.ravel(a), np.ravel(b)))


@pytest.fixture(scope="module", params=[0.0, 0.3])
def small(request):
    mu = request.param
    dims = (2, 2, 4, 4)
    lat, u = make_lattice(dims, 0.8, seed=0)
    xs = latgen.random_sources(dims, 2, 1)
    dov = O.dense_dov(D.sign_schur(W.dense_matrix(u, M_W, mu)))
    yield mu, lat, xs, dov
    lat.close()


@pytest.mark.parametrize("dagger", [False, True])
def test_apply_matches_dense(small, dagger):
    mu, lat, xs, dov = small
    banner(f"overlap apply 2x2x4x4 mu={mu} dagger={dagger} k=400")
    y, rc = _apply(lat, xs[0], dagger, mu=mu, k=400, ell=0)
    ref = (dov.conj().T if dagger else dov) @ xs[0].reshape(-1)
    assert rc == 0
    assert rel(y, ref) < 1e-9


def test_solve_matches_dense(small):
    mu, lat, xs, dov = small
    banner(f"overlap CGNR 2x2x4x4 mu={mu} k=400")
    b = nk()
    db = to_dev(xs[1])
    dy = torch_cuda().empty_like(db)
    it, res, rc = b.nk_overlap_solve_device(lat.h, _params(mu=mu, k=400, ell=0), 1e-11, 100, db, dy)
    assert rc == 0 and res <= 1e-11 and 5 <= it <= 40
    y = to_host(dy)
    assert rel(y, np.linalg.solve(dov, xs[1].reshape(-1))) < 1e-9
    # the oracle's CGNR on the dense operator takes about as many steps
    _, it_o, _, _ = O.cgnr(lambda v: dov @ v, lambda v: dov.conj().T @ v, xs[1].reshape(-1), 1e-11, 100)
    assert abs(it - it_o) <= 2


def test_solve_edge_cases(small):
    mu, lat, xs, dov = small
    b = nk()
    p = _params(mu=mu, k=200, ell=0)
    db = to_dev(np.zeros_like(xs[0]))
    dy = torch_cuda().empty_like(db)
    dy.fill_(1.0)
    it, res, rc = b.nk_overlap_solve_device(lat.h, p, 1e-8, 10, db, dy)
    assert (it, rc) == (0, 0) and not np.any(to_host(dy))
    db = to_dev(xs[0])
    it, res, rc = b.nk_overlap_solve_device(lat.h, p, 1e-12, 1, db, dy)
    assert it == 1 and rc == b.NK_WARN_NOTCONV and 0 < res < 1
    for bad in (dict(tol=0.0, maxit=10), dict(tol=1e-8, maxit=0)):
        with pytest.raises(b.NKError) as ei:
            b.nk_overlap_solve_device(lat.h, p, bad["tol"], bad["maxit"], db, dy)
        assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_overlap_solve_device(lat.h, _params(mu=mu, k=200, ell=0, nrhs=2), 1e-8, 10,
                                  to_dev(xs), torch_cuda().empty_like(to_dev(xs)))
    assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_overlap_apply_device(lat.h, p, False, db, db)
    assert ei.value.code == b.NK_EINVAL


@pytest.fixture(scope="module")
def big():
    dims = (16, 16, 16, 16)
    lat, u = make_lattice(dims, 0.8, seed=0)
    xs = latgen.random_sources(dims, 2, 0)
    yield lat, xs
    lat.close()


def test_full_size_adjoint_and_ginsparg_wilson(big):
    lat, xs = big
    banner("overlap 16^4 mu=0.3 k=500 l=60: adjoint and Ginsparg-Wilson")
    kw = dict(mu=0.3, k=500, ell=60)
    u, v = xs
    dv, _ = _apply(lat, v, False, **kw)
    du, _ = _apply(lat, u, True, **kw)
    lhs, rhs = _cdot(u, dv), _cdot(du, v)
    scale = np.linalg.norm(u) * np.linalg.norm(v)
    assert abs(lhs - rhs) < 1e-7 * scale
    g5v = O.gamma5(v)
    a, _ = _apply(lat, g5v, False, **kw)  # Dov g5 v
    gw_l = O.gamma5(dv) + a  # g5 Dov v + Dov g5 v
    gw_r, _ = _apply(lat, O.gamma5(dv.reshape(v.shape)), False, **kw)  # Dov g5 Dov v
    assert rel(gw_l, gw_r) < 1e-7


def test_full_size_solve(big):
    lat, xs = big
    banner("overlap CGNR 16^4 mu=0.3 k=500 l=60 tol=1e-7")
    b = nk()
    kw = dict(mu=0.3, k=500, ell=60)
    db = to_dev(xs[0])
    dy = torch_cuda().empty_like(db)
    it, res, rc = b.nk_overlap_solve_device(lat.h, _params(**kw), 1e-7, 100, db, dy)
    assert rc == 0 and res <= 1e-7 and it < 60
    dr, _ = _apply(lat, to_host(dy).reshape(xs[0].shape), False, **kw)
    assert rel(dr, xs[0]) < 1e-6


def test_deflated_overlap_and_solve(small):
    """Dov and Dov^dag with the sign deflated by 16 critical eigenpairs of A
    (Dov^dag uses the eigenpairs of A^dag these give: conj(lambda), L, R), at
    k = 200 where the undeflated operator is still far off; and CGNR with it."""
    from oracle import deflation as DF

    mu, lat, xs, dov = small
    banner(f"deflated overlap 2x2x4x4 mu={mu} k=200 m=16")
    b = nk()
    u = latgen.random_gauge((2, 2, 4, 4), 0.8, 0)
    lam, r, l = DF.critical_eigenpairs(W.dense_matrix(u, M_W, mu), 16, mu == 0.0)
    R, L = to_dev(r.T), to_dev(l.T)
    p = _params(mu=mu, k=200, ell=0)
    dx = to_dev(xs[0])
    dy = torch_cuda().empty_like(dx)
    for dagger in (False, True):
        ref = (dov.conj().T if dagger else dov) @ xs[0].reshape(-1)
        b.nk_overlap_apply_device(lat.h, p, dagger, dx, dy, lam=lam, R=R, L=L)
        e_d = rel(to_host(dy), ref)
        b.nk_overlap_apply_device(lat.h, p, dagger, dx, dy)
        e_p = rel(to_host(dy), ref)
        assert e_d < 1e-8 and e_p > 100 * e_d, (dagger, e_d, e_p)
    db = to_dev(xs[1])
    it, res, rc = b.nk_overlap_solve_device(lat.h, p, 1e-9, 100, db, dy, lam=lam, R=R, L=L)
    assert rc == 0 and res <= 1e-9
    assert rel(to_host(dy), np.linalg.solve(dov, xs[1].reshape(-1))) < 1e-8
    with pytest.raises(b.NKError) as ei:
        b.nk_overlap_apply_device(lat.h, p, False, dx, R[: dx.numel()], lam=lam, R=R, L=L)
    assert ei.value.code == b.NK_EINVAL


def test_overlap_spectrum_on_the_circle_mu0():
    """At mu = 0 the eigenvalues of Dov lie on |z - 1| = 1 (Sec. 1, Eq. (1)):
    Dov - 1 = gamma5 sgn(H) with H = gamma5 Dw(0) Hermitian is unitary and Dov
    is normal.  On the benchmark lattice (16^4, link width 0.8, k = 500,
    l = 60): |(Dov - 1) x| = |x| and Dov^dag Dov x = Dov Dov^dag x for
    Gaussian x, to the sign's accuracy there (3.5e-10, bound 1e-8); and on
    the 16 eigenvectors r_i of H smallest in modulus from the library's
    eigensolver, with the sign deflated by them, (Dov - 1) r_i = sgn(lambda_i)
    gamma5 r_i, so |Dov r_i - 1 r_i| = 1 and <gamma5 r_j, (Dov - 1) r_i> =
    sgn(lambda_i) delta_ij, to the eigenvectors' accuracy (1e-8)."""
    b = nk()
    torch = torch_cuda()
    dims = (16, 16, 16, 16)
    lat, u = make_lattice(dims, 0.8, seed=0)
    kw = dict(mu=0.0, k=500, ell=60)
    xs = latgen.random_sources(dims, 2, 12)
    banner("overlap spectrum 16^4 mu=0: unitarity of Dov - 1 and normality")
    for x in xs:
        y, _ = _apply(lat, x, False, **kw)
        assert abs(np.linalg.norm(y - x.reshape(-1)) / np.linalg.norm(x) - 1.0) < 1e-8
        yd, _ = _apply(lat, x, True, **kw)
        a1, _ = _apply(lat, yd.reshape(x.shape), False, **kw)  # Dov Dov^dag x
        a2, _ = _apply(lat, y.reshape(x.shape), True, **kw)    # Dov^dag Dov x
        assert rel(a1, a2) < 1e-8
    banner("overlap spectrum 16^4 mu=0: deflated, on the eigensolver's eigenvectors")
    m, p = 16, 32  # the benchmark's setting: converges in 36 passes on this lattice
    V0 = to_dev(latgen.random_sources(dims, p, 11))
    R = torch.empty(m * 12 * 16 ** 4, dtype=torch.complex128, device="cuda")
    lam, passes, res, rc = b.nk_eig_hermitian_device(lat.h, M_W, m, p, 40, 1e-10, 100, V0, R)
    assert rc == 0
    lamc = lam.astype(np.complex128)
    rh = to_host(R).reshape(m, -1)
    g5 = np.tile(np.repeat(O.G5, 3), 16 ** 4)
    out = torch.empty_like(R)
    b.nk_overlap_apply_device(lat.h, _params(nrhs=m, **kw), False, R, out, lam=lamc, R=R, L=R)
    dov_r = to_host(out).reshape(m, -1)
    gram = np.array([[np.vdot(g5 * rh[j], dov_r[i] - rh[i]) for i in range(m)] for j in range(m)])
    print(f"[spectrum] |Dov r - r| = {[round(float(np.linalg.norm(dov_r[i] - rh[i])), 12) for i in range(m)]}",
          flush=True)
    assert np.allclose(np.abs(np.diag(gram)), 1.0, atol=1e-8)
    assert np.allclose(np.diag(gram).real, np.sign(lam), atol=1e-8)
    assert np.max(np.abs(gram - np.diag(np.diag(gram)))) < 1e-8
    lat.close()
