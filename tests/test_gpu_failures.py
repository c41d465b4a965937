"""Failure handling through the C ABI: every case is an input the library
turns into a return code before or during ordinary kernel work (no kernel is
made to fault).

* Roberts-Higham on a matrix with a purely imaginary eigenvalue: the scalar
  map sends z = i to (i + 1/i) / 2 = 0 exactly, so the next inversion meets a
  zero pivot (R11: sgn is undefined there) -> NK_WARN_NOTCONV;
* the iteration cap reached before the stopping test -> NK_WARN_NOTCONV;
* a source with a NaN -> NK_EINVAL;
* V_k larger than the device with two-pass lifting switched off -> NK_ENOMEM;
* a serious breakdown of two-sided Lanczos at its first step (a free-field
  plane wave times a spinor with w_hat^dag v_hat = 0) -> NK_WARN_BREAKDOWN and
  the result of the steps before it, alone and next to an ordinary source in
  a lockstep run;
* and the exact case at the other end: a source that is an eigenvector of
  gamma5 Dw(mu) (a free-field plane wave) comes back as sgn(Re lambda) x.
"""
import numpy as np
import pytest

import latgen
from oracle import freefield as F
from oracle import krylov as K
from oracle import nested as N
from oracle import wilson as W
from tests import breakdown_source as BS
from tests.gpu_helpers import M_W, banner, make_lattice, nk, rel, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _diag_with_imaginary(n, seed):
    """A diagonal matrix with one eigenvalue exactly i, conjugated by a
    permutation (exact in floating point), so the iteration reaches the
    zero pivot bit for bit."""
    rng = np.random.default_rng(seed)
    d = np.where(rng.random(n) < 0.5, -1.0, 1.0) * (0.5 + rng.random(n)) + 0j
    d[n // 3] = 1j
    perm = rng.permutation(n)
    a = np.zeros((n, n), np.complex128)
    a[perm, perm] = d
    return a


@pytest.mark.parametrize("n", [3, 97, 200])
def test_rh_purely_imaginary_eigenvalue_warns(n):
    banner(f"rh with an eigenvalue i, n={n}")
    b = nk()
    a = _diag_with_imaginary(n, n)
    _, _, rc = b.nk_rh_sign(a)
    assert rc == b.NK_WARN_NOTCONV
    assert "singular" in b.nk_last_error()


@pytest.mark.parametrize("n", [50, 200])
def test_rh_iteration_cap_warns(n):
    banner(f"rh iteration cap, n={n}")
    b = nk()
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a += 3.0 * np.diag(np.where(rng.random(n) < 0.5, -1.0, 1.0))
    _, it, rc = b.nk_rh_sign(a, maxit=2)
    assert rc == b.NK_WARN_NOTCONV and int(it[0]) == 2
    assert "did not converge" in b.nk_last_error()
    _, it, rc = b.nk_rh_sign(a)
    assert rc == b.NK_OK and 2 < int(it[0]) < 100


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_nan_source_is_an_error(mu):
    b = nk()
    dims = (4, 4, 2, 6)
    lat, _ = make_lattice(dims, 0.6, seed=3)
    x = latgen.random_sources(dims, 1, 4)[0]
    x.reshape(-1)[17] = np.nan
    banner(f"NaN source, mu={mu}")
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=40, ell=10, mu=mu), dx, dy)
    assert ei.value.code == b.NK_EINVAL
    assert "non-finite" in b.nk_last_error()
    lat.close()


def test_basis_too_large_without_two_pass_is_enomem():
    """(k + 1) columns of 12.6 MB at 16^4 for k = 30000 exceed any MI355X;
    with two_pass = OFF the call refuses before allocating."""
    b = nk()
    dims = (16, 16, 16, 16)
    lat, _ = make_lattice(dims, 0.8, seed=0)
    x = latgen.random_sources(dims, 1, 0)[0]
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    banner("V_k too large, two_pass off")
    p = b.nk_sign_params_default(k=30000, ell=0, mu=0.3, two_pass=b.NK_TWO_PASS_OFF)
    with pytest.raises(b.NKError) as ei:
        b.nk_sign_apply_device(lat.h, p, dx, dy)
    assert ei.value.code == b.NK_ENOMEM
    assert "two_pass is OFF" in b.nk_last_error()
    lat.close()


def _plane_wave_eigenvector(dims, mu, n, which):
    """exp(i p.x) s (colour 0) with s the `which`-th eigenvector of the 4 x 4
    gamma5 Dw(p) at momentum index n = (nx, ny, nz, nt); returns (psi, lambda)."""
    lx, ly, lz, lt = dims
    mats = F.g5dw_momentum(dims, M_W, mu)
    nx, ny, nz, nt = n
    lam, vec = np.linalg.eig(mats[nt, nz, ny, nx])
    s = vec[:, which] / np.linalg.norm(vec[:, which])
    px, py, pz, pt = F.momenta(dims)
    x = np.arange(lx)[None, None, None, :]
    y = np.arange(ly)[None, None, :, None]
    z = np.arange(lz)[None, :, None, None]
    t = np.arange(lt)[:, None, None, None]
    phase = np.exp(1j * (px[0, 0, 0, nx] * x + py[0, 0, ny, 0] * y + pz[0, nz, 0, 0] * z + pt[nt, 0, 0, 0] * t))
    psi = np.zeros((lt, lz, ly, lx, 4, 3), np.complex128)
    psi[..., :, 0] = phase[..., None] * s
    return psi, lam[which]


@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("ell", [0, 6])
def test_eigenvector_source_gives_sign_of_its_eigenvalue(mu, ell):
    """A free-field plane wave times an eigenvector of gamma5 Dw(p) spans an
    invariant subspace of dimension one: the method returns sgn(Re lambda) x
    (the recurrence continues through directions of rounding size that the
    small problem decouples)."""
    b = nk()
    dims = (4, 4, 4, 8)
    lat, _ = make_lattice(dims, 0.0, unit=True)
    for n, which in (((1, 0, 2, 3), 0), ((0, 3, 1, 5), 2)):
        psi, lam = _plane_wave_eigenvector(dims, mu, n, which)
        # the plane wave really is an eigenvector of the operator
        assert rel(F.g5dw_apply_free(psi, M_W, mu), lam * psi) < 1e-13
        banner(f"eigenvector source mu={mu} ell={ell} p={n} lambda={lam:.4f}")
        dx = to_dev(psi)
        dy = torch_cuda().empty_like(dx)
        b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=30, ell=ell, mu=mu), dx, dy)
        y = to_host(dy)
        assert rel(y, np.sign(lam.real) * psi.reshape(-1)) < 1e-10, (n, lam)
    lat.close()


def _breakdown_case(mu):
    """(x, y_ref): the breakdown source and the oracle's result from its one
    basis vector, sgn(Re alpha_0) x."""
    s, r = BS.breakdown_spinor(M_W, mu)
    assert r < 1e-14
    x = BS.plane_wave(s)
    u = latgen.unit_gauge(BS.DIMS)
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -mu).reshape(-1)
    kr = K.two_sided_lanczos(f, fd, x.reshape(-1), 20)
    assert kr.breakdown == 1 and kr.H.k == 1
    z, _ = N.small_sign(kr.H, 0, False)
    y = kr.norm_x * kr.V @ z
    assert rel(y, np.sign(kr.H.alpha[0].real) * x.reshape(-1)) < 1e-13
    return x, y


@pytest.mark.parametrize("mu", [0.3, 0.5])
@pytest.mark.parametrize("ell", [0, 4])
def test_two_sided_serious_breakdown(mu, ell):
    b = nk()
    x, yref = _breakdown_case(mu)
    lat, _ = make_lattice(BS.DIMS, 0.0, unit=True)
    banner(f"2sL serious breakdown at step 1, mu={mu} ell={ell}")
    dx = to_dev(x)
    dy = torch_cuda().empty_like(dx)
    info, rc = b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=20, ell=ell, mu=mu), dx, dy)
    assert rc == b.NK_WARN_BREAKDOWN
    assert info.breakdown_step == 1 and info.k_used == 1
    assert rel(to_host(dy), yref) < 1e-12
    lat.close()


def test_lockstep_breakdown_leaves_the_other_source_alone():
    """block = 1 with the breakdown source beside a Gaussian one: the first
    stops after one step, the second runs all k steps and agrees with its
    own single-source run."""
    b = nk()
    mu, k, ell = 0.3, 24, 6
    x0, y0ref = _breakdown_case(mu)
    x1 = latgen.random_sources(BS.DIMS, 1, 11)[0]
    lat, _ = make_lattice(BS.DIMS, 0.0, unit=True)
    torch = torch_cuda()
    banner("lockstep: breakdown source next to a Gaussian source")
    d1 = to_dev(x1)
    y1 = torch.empty_like(d1)
    _, rc1 = b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=k, ell=ell, mu=mu), d1, y1)
    assert rc1 == b.NK_OK
    xb = to_dev(np.stack([x0, x1]))
    yb = torch.empty_like(xb)
    info, rc = b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=k, ell=ell, mu=mu, nrhs=2, block=1), xb, yb)
    assert rc == b.NK_WARN_BREAKDOWN and info.breakdown_step == 1
    ybh = to_host(yb).reshape(2, -1)
    assert rel(ybh[0], y0ref) < 1e-12
    assert rel(ybh[1], to_host(y1)) < 1e-9
    lat.close()


def test_destroyed_handles_and_host_calls_free_their_device_memory():
    """A cycle of handle create, host-pointer application, lockstep run and
    destroy, twice: the second cycle ends with as much free device memory as
    the first (the library's file-scope workspaces are sized by the first)."""
    b = nk()
    torch = torch_cuda()
    dims = (8, 8, 8, 8)
    u = latgen.random_gauge(dims, 0.6, 2)
    xs = latgen.random_sources(dims, 2, 3)

    def cycle():
        lat = b.Lattice(dims)
        b.nk_gauge_set(lat.h, u)
        y = np.empty_like(xs[0].reshape(-1))
        info = b.nk_sign_info()
        p = b.nk_sign_params_default(k=60, ell=20, mu=0.3)
        rc = b.library().nk_sign_apply(lat.h, b.C.byref(p), b._hptr(np.ascontiguousarray(xs[0].reshape(-1))),
                                       b._hptr(y), b.C.byref(info))
        assert rc == b.NK_OK
        dx = to_dev(xs)
        dy = torch.empty_like(dx)
        _, rc = b.nk_sign_apply_device(lat.h, b.nk_sign_params_default(k=60, ell=20, mu=0.3, nrhs=2, block=1), dx, dy)
        assert rc == b.NK_OK
        del dx, dy
        lat.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return torch.cuda.mem_get_info()[0]

    banner("handle create/apply/destroy twice: no device memory kept")
    f1 = cycle()
    f2 = cycle()
    assert f2 >= f1 - (16 << 20), (f1, f2)
