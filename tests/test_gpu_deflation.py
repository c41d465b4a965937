"""GPU parity of the deflated sign (Sec. 2, critical eigenvalues treated exactly).

* method level, small lattice: nk_sign_apply_deflated_device against the
  oracle's deflated run at the same (k, l) with the same eigenpairs (dense
  eigen-decomposition), within method_bound (the oracle's own rounding
  sensitivity) as for the undeflated
  method, and against the exact sign;
* the exact part alone: every eigenpair deflated (nothing left for the Krylov
  part) reproduces the spectral sign to 1e-10;
* full size, 16^4 free field: exact plane-wave eigenpairs (checked on the CPU
  against the oracle's stencil first); a source in their span comes out exact,
  and a general source matches the momentum-space closed form;
* edge cases: m = 0 is the undeflated call bit for bit, a zero source in a
  batch gets y = 0 and leaves the other source's bits alone, lockstep sources
  agree with one at a time, invalid arguments are rejected.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import latgen
from oracle import deflation as DF
from oracle import dense as D
from oracle import freefield as FF
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, make_lattice, method_bound, nk, perturbed, rel, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _run(lat, x, lam, r, l, nrhs=1, **kw):
    b = nk()
    p = b.nk_sign_params_default(nrhs=nrhs, **kw)
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    info, rc = b.nk_sign_apply_deflated_device(lat.h, p, lam, to_dev(r.T), to_dev(l.T), dx, dy)
    return to_host(dy), info, rc


def _ops(u, shape, mu):
    f = lambda v: W.a_apply(u, v.reshape(shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(shape), M_W, -mu).reshape(-1)
    return f, fd


@pytest.fixture(scope="module", params=[0.0, 0.3])
def small(request):
    mu = request.param
    dims = (2, 2, 4, 4)
    lat, u = make_lattice(dims, 0.8, seed=0)
    x = latgen.random_sources(dims, 1, 0)[0]
    a = W.dense_matrix(u, M_W, mu)
    lam, r, l = DF.critical_eigenpairs(a, 16, mu == 0.0)
    exact = D.sign_spectral(a, hermitian=mu == 0.0) @ x.reshape(-1)
    yield mu, lat, u, x, lam, r, l, exact
    lat.close()


@pytest.mark.parametrize("ell", [0, 40])
def test_deflated_matches_oracle(small, ell):
    mu, lat, u, x, lam, r, l, exact = small
    banner(f"deflation 2x2x4x4 mu={mu} k=80 ell={ell} m=16")
    f, fd = _ops(u, x.shape, mu)
    yo, _ = DF.deflated_sign_apply(f, fd, x, 80, ell, mu == 0.0, lam, r, l)
    y, info, rc = _run(lat, x, lam, r, l, mu=mu, k=80, ell=ell)
    eps_true = rel(yo, exact)
    assert rc == 0
    sens = rel(DF.deflated_sign_apply(f, fd, perturbed(x), 80, ell, mu == 0.0, lam, r, l)[0], yo)
    print(f"[gap] deflated: GPU vs oracle {rel(y, yo):.3e}, sensitivity {sens:.3e}", flush=True)
    assert rel(y, yo) <= method_bound(sens)
    assert rel(y, exact) < 2 * eps_true + 1e-12
    # and deflation pays: the undeflated GPU run at the same k is further off
    b = nk()
    p = b.nk_sign_params_default(mu=mu, k=80, ell=ell)
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    b.nk_sign_apply_device(lat.h, p, dx, dy)
    assert rel(to_host(dy), exact) > 5 * rel(y, exact)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_deflation_is_the_spectral_sign(mu):
    dims = (2, 2, 2, 2)
    banner(f"deflation 2^4 mu={mu}: all 192 eigenpairs")
    lat, u = make_lattice(dims, 1.0, seed=3)
    x = latgen.random_sources(dims, 1, 3)[0]
    a = W.dense_matrix(u, M_W, mu)
    lam, r, l = DF.critical_eigenpairs(a, a.shape[0], mu == 0.0)
    y, info, rc = _run(lat, x, lam, r, l, mu=mu, k=8, ell=0)
    assert rc == 0
    assert rel(y, D.sign_schur(a) @ x.reshape(-1)) < 1e-10
    lat.close()


def test_no_deflation_is_the_undeflated_call(small):
    mu, lat, u, x, lam, r, l, exact = small
    banner(f"deflation m=0 mu={mu}")
    b = nk()
    p = b.nk_sign_params_default(mu=mu, k=60, ell=30)
    dx = to_dev(x)
    y0 = torch_cuda().empty_like(dx)
    y1 = torch_cuda().empty_like(dx)
    b.nk_sign_apply_device(lat.h, p, dx, y0)
    e = torch_cuda().empty(0, dtype=dx.dtype, device=dx.device)
    b.nk_sign_apply_deflated_device(lat.h, p, np.zeros(0, np.complex128), e, e, dx, y1)
    assert np.array_equal(to_host(y0), to_host(y1))


def test_zero_source_and_batch(small):
    mu, lat, u, x, lam, r, l, exact = small
    banner(f"deflation zero source in a batch, lockstep batch, mu={mu}")
    y1, _, rc1 = _run(lat, x, lam, r, l, mu=mu, k=60, ell=30)
    pair = np.stack([np.zeros_like(x), x])
    y2, _, rc2 = _run(lat, pair, lam, r, l, nrhs=2, mu=mu, k=60, ell=30)
    y2 = y2.reshape(2, -1)
    assert rc1 == 0 and rc2 == 0
    assert not np.any(y2[0])
    assert np.array_equal(y2[1], y1)
    # three live sources in lockstep against one at a time
    xs = latgen.random_sources(x.shape[:4][::-1], 3, 5)
    yb, _, rcb = _run(lat, xs, lam, r, l, nrhs=3, mu=mu, k=60, ell=30, block=1)
    yb = yb.reshape(3, -1)
    for s in range(3):
        ys, _, _ = _run(lat, xs[s], lam, r, l, mu=mu, k=60, ell=30)
        assert rel(yb[s], ys) < 1e-9  # other reduction order, as for the undeflated lockstep path


def test_invalid_arguments(small):
    mu, lat, u, x, lam, r, l, exact = small
    b = nk()
    p = b.nk_sign_params_default(mu=mu, k=40, ell=10)
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    R, L = to_dev(r.T), to_dev(l.T)
    bad = lam.copy()
    bad[2] = 1j * abs(bad[2])
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_deflated_device(lat.h, p, bad, R, L, dx, dy)
    assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_deflated_device(lat.h, p, np.ones(b.NK_DEFL_MAX + 1, np.complex128), R, L, dx, dy)
    assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_deflated_device(lat.h, p, lam, R, L, dx, dx)
    assert ei.value.code == b.NK_EINVAL
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_deflated_device(lat.h, p, lam, R, L, dx, R[: dx.numel()])
    assert ei.value.code == b.NK_EINVAL


def _free_eigenpairs(dims, mu, nmom):
    """Exact eigenpairs of the free operator: plane waves of the nmom momenta
    whose 4 x 4 matrices have the eigenvalues closest to the imaginary axis,
    times every spin eigenvector and colour; columns of R and L, L^dag R = I."""
    mats = FF.g5dw_momentum(dims, M_W, mu)  # (Lt, Lz, Ly, Lx, 4, 4)
    ev = np.linalg.eigvals(mats.reshape(-1, 4, 4))
    order = np.argsort(np.abs(ev.real).min(axis=1), kind="stable")[:nmom]
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    t, z, y_, x_ = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    lams, rs, ls = [], [], []
    for flat in order:
        it, iz, iy, ix = np.unravel_index(flat, (lt, lz, ly, lx))
        p = (2 * np.pi * ix / lx, 2 * np.pi * iy / ly, 2 * np.pi * iz / lz, (2 * it + 1) * np.pi / lt)
        pw = np.exp(1j * (p[0] * x_ + p[1] * y_ + p[2] * z + p[3] * t)) / np.sqrt(V)
        w, zl, xr = sla.eig(mats[it, iz, iy, ix], left=True, right=True)
        zl = zl @ np.linalg.inv(zl.conj().T @ xr).conj().T
        for s in range(4):
            for c in range(3):
                e = np.zeros((4, 3), np.complex128)
                e[:, c] = xr[:, s]
                rs.append((pw[..., None, None] * e).reshape(-1))
                e = np.zeros((4, 3), np.complex128)
                e[:, c] = zl[:, s]
                ls.append((pw[..., None, None] * e).reshape(-1))
                lams.append(w[s])
    return np.array(lams), np.stack(rs, axis=1), np.stack(ls, axis=1)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_size_free_field(mu):
    dims = (16, 16, 16, 16)
    banner(f"deflation 16^4 free field mu={mu}: 2 momenta, m=24")
    lam, r, l = _free_eigenpairs(dims, mu, 2)
    u1 = latgen.unit_gauge(dims)
    shape = (16, 16, 16, 16, 4, 3)
    for i in (0, 13):  # eigenpairs, checked against the oracle's position-space stencil
        ar = W.a_apply(u1, r[:, i].reshape(shape), M_W, mu).reshape(-1)
        assert np.linalg.norm(ar - lam[i] * r[:, i]) < 1e-12 * abs(lam[i]) * np.linalg.norm(r[:, i])
        al = W.a_apply(u1, l[:, i].reshape(shape), M_W, -mu).reshape(-1)
        assert np.linalg.norm(al - np.conj(lam[i]) * l[:, i]) < 1e-12 * abs(lam[i]) * np.linalg.norm(l[:, i])
    assert np.linalg.norm(l.conj().T @ r - np.eye(len(lam))) < 1e-12
    lat, _ = make_lattice(dims, 0.0, unit=True)
    # a source in the span of the deflated eigenvectors comes out exact
    a = latgen.random_sources((4, 3, 2, 1), 1, 7).reshape(-1)[: len(lam)]
    xs = r @ a
    y, info, rc = _run(lat, xs, lam, r, l, mu=mu, k=20, ell=10)
    assert rc == 0
    assert rel(y, r @ (np.sign(lam.real) * a)) < 1e-12
    # a general source matches the closed form
    x = latgen.random_sources(dims, 1, 3)[0]
    y, info, rc = _run(lat, x, lam, r, l, mu=mu, k=330, ell=150)
    assert rc == 0
    assert rel(y, FF.sign_apply_free(x, M_W, mu)) < 1e-10
    lat.close()


def test_python_convenience_wrapper(small):
    mu, lat, u, x, lam, r, l, exact = small
    banner(f"nk.sign_apply_deflated mu={mu}")
    b = nk()
    y1, _, rc1 = _run(lat, x, lam, r, l, mu=mu, m_w=M_W, k=60, ell=30)
    y2, info = b.sign_apply_deflated(lat, to_dev(x), lam, to_dev(r.T), to_dev(l.T), mu=mu, m_w=M_W, k=60, ell=30)
    assert info.rc == rc1 == 0
    assert np.array_equal(to_host(y2), y1)
    with pytest.raises(ValueError):
        b.sign_apply_deflated(lat, to_dev(x), lam[:3], to_dev(r.T), to_dev(l.T), mu=mu, k=60, ell=30)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_deflation_lowers_k_at_1e8(mu):
    """What deflation is for: the smallest k (on a grid of 20, l = k/4) whose
    nested result is within 1e-8 of the exact sign, with and without the 16
    critical eigenpairs deflated.  The oracle's scan on this lattice gives
    240 -> 200 at mu = 0 and 300 -> 240 at mu = 0.3."""
    dims = (2, 4, 4, 4)
    banner(f"deflation 2x4x4x4 mu={mu}: smallest k at 1e-8, m = 16 against none")
    lat, u = make_lattice(dims, 0.8, seed=0)
    x = latgen.random_sources(dims, 1, 0)[0]
    a = W.dense_matrix(u, M_W, mu)
    lam, r, l = DF.critical_eigenpairs(a, 16, mu == 0.0)
    exact = D.sign_schur(a) @ x.reshape(-1)
    b = nk()
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    R, L = to_dev(r.T), to_dev(l.T)
    err_p, err_d = {}, {}
    for k in range(160, 341, 20):
        p = b.nk_sign_params_default(mu=mu, m_w=M_W, k=k, ell=k // 4)
        b.nk_sign_apply_device(lat.h, p, dx, dy)
        err_p[k] = rel(to_host(dy), exact)
        b.nk_sign_apply_deflated_device(lat.h, p, lam, R, L, dx, dy)
        err_d[k] = rel(to_host(dy), exact)
    k_p = min(k for k, e in err_p.items() if e < 1e-8)
    k_d = min(k for k, e in err_d.items() if e < 1e-8)
    print(f"mu={mu}: k at 1e-8 undeflated {k_p}, deflated {k_d};",
          " ".join(f"{k}:{err_p[k]:.1e}/{err_d[k]:.1e}" for k in sorted(err_p)), flush=True)
    assert k_d < k_p
    lat.close()


def test_graph_replays_and_reduced_precision(small):
    """The deflated path under the other execution modes it passes through:
    lockstep sweeps replayed from captured graphs (block = 2) agree with one
    source at a time, and FP32 spinors and links stay within the reduced
    precision's error of the FP64 deflated result."""
    mu, lat, u, x, lam, r, l, exact = small
    banner(f"deflation with graph replays and FP32, mu={mu}")
    xs = latgen.random_sources(x.shape[:4][::-1], 3, 9)
    yb, _, rcb = _run(lat, xs, lam, r, l, nrhs=3, mu=mu, k=60, ell=30, block=2)
    yb2, _, _ = _run(lat, xs, lam, r, l, nrhs=3, mu=mu, k=60, ell=30, block=2)  # replays the captured graphs
    yb, yb2 = yb.reshape(3, -1), yb2.reshape(3, -1)
    assert np.array_equal(yb, yb2)
    for s in range(3):
        ys, _, _ = _run(lat, xs[s], lam, r, l, mu=mu, k=60, ell=30)
        assert rel(yb[s], ys) < 1e-9
    y64, _, _ = _run(lat, x, lam, r, l, mu=mu, k=80, ell=40)
    y32, _, _ = _run(lat, x, lam, r, l, mu=mu, k=80, ell=40, precision=1)
    assert rel(y32, y64) < 1e-5
