"""GPU parity of the Wilson stencil gamma5 Dw(mu) (Sec. 1) against the oracle.

Element-by-element against the oracle's Dw on several lattices (including the
smallest even extents, where forward and backward neighbours coincide, and a
shape with all extents different), and at the full 16^4 size against the
free-field closed form and the gamma5-hermiticity identity, in the launch
configuration the benchmark uses.  FP64 tolerance 1e-14 relative (the stencil
is a fixed sum of at most 8 x 2 x 9 products; rounding is a few ulp).
"""
import numpy as np
import pytest

import latgen
from oracle import freefield as F
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, make_lattice, nk, rel, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (6, 4, 2, 10)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("g5", [True, False])
def test_apply_dw_matches_oracle(dims, mu, g5):
    banner(f"apply_dw dims={dims} mu={mu} g5={g5}")
    lat, u = make_lattice(dims, 0.8, seed=3)
    b = nk()
    x = latgen.random_sources(dims, 2, 4)
    y = b.nk_apply_dw(lat.h, M_W, mu, g5, x.reshape(-1), nrhs=2)
    for r in range(2):
        ref = W.dw_apply(u, x[r], M_W, mu, g5=g5)
        assert rel(y.reshape(2, -1)[r], ref) < TOL * 10
    lat.close()


@pytest.mark.parametrize("mu", [0.0, 0.5])
def test_pair_matches_oracle(mu):
    dims = (4, 2, 6, 4)
    banner(f"apply_pair dims={dims} mu={mu}")
    lat, u = make_lattice(dims, 1.0, seed=7)
    b = nk()
    v, w = latgen.random_sources(dims, 2, 8)
    dv, dw = to_dev(v), to_dev(w)
    torch = torch_cuda()
    av = torch.empty_like(dv)
    adw = torch.empty_like(dw)
    b.nk_apply_pair_device(lat.h, M_W, mu, dv, dw, av, adw)
    torch.cuda.synchronize()
    assert rel(to_host(av), W.a_apply(u, v, M_W, mu)) < TOL * 10
    assert rel(to_host(adw), W.a_dag_apply(u, w, M_W, mu)) < TOL * 10
    lat.close()


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_size_free_field(mu):
    dims = (16, 16, 16, 16)
    banner(f"free field 16^4 mu={mu}")
    lat, _ = make_lattice(dims, 0.0, unit=True)
    b = nk()
    x = latgen.random_sources(dims, 1, 1)[0]
    dx = to_dev(x)
    torch = torch_cuda()
    dy = torch.empty_like(dx)
    b.nk_apply_dw_device(lat.h, M_W, mu, True, dx, dy)
    torch.cuda.synchronize()
    assert rel(to_host(dy), F.g5dw_apply_free(x, M_W, mu)) < TOL * 10
    lat.close()


def test_full_size_gamma5_hermiticity_and_samples():
    dims = (16, 16, 16, 16)
    mu = 0.3
    banner("16^4 eps=0.8: <y, A(mu) x> = <A(-mu) y, x>, sampled sites vs oracle")
    lat, u = make_lattice(dims, 0.8, seed=0)
    b = nk()
    x, y = latgen.random_sources(dims, 2, 2)
    torch = torch_cuda()
    dx, dy = to_dev(x), to_dev(y)
    ax, ay = torch.empty_like(dx), torch.empty_like(dy)
    b.nk_apply_dw_device(lat.h, M_W, mu, True, dx, ax)
    b.nk_apply_dw_device(lat.h, M_W, -mu, True, dy, ay)
    torch.cuda.synchronize()
    lhs = torch.vdot(dy, ax).item()
    rhs = torch.vdot(ay, dx).item()
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # sampled sites against the oracle's full application
    ref = W.dw_apply(u, x, M_W, mu, g5=True)
    got = to_host(ax).reshape(ref.shape)
    rng = np.random.default_rng(0)
    for _ in range(64):
        t, z, yy, xx = (int(v) for v in rng.integers(0, 16, 4))
        assert np.max(np.abs(got[t, z, yy, xx] - ref[t, z, yy, xx])) < 1e-13 * np.max(np.abs(ref))
    assert rel(got, ref) < TOL * 10
    lat.close()


def test_apply_without_gauge_is_an_error():
    b = nk()
    lat = b.Lattice((2, 2, 2, 2))
    x = np.zeros(12 * 16, np.complex128)
    with pytest.raises(b.NKError) as ei:
        b.nk_apply_dw(lat.h, M_W, 0.0, True, x)
    assert ei.value.code == b.NK_ENOGAUGE
    lat.close()


@pytest.mark.parametrize("dims", [(2, 4, 6, 8), (16, 16, 16, 16)])
def test_packed_layout_round_trip_and_repeated_application(dims):
    """Packing is a permutation (the round trip is exact and inner products
    agree); the packed applications give the same bits as the canonical entry
    points; two applications in the packed layout match the oracle's A(A x)
    (sampled sites at 16^4)."""
    mu = 0.3
    banner(f"packed layout dims={dims} mu={mu}")
    lat, u = make_lattice(dims, 0.8, seed=2)
    b = nk()
    torch = torch_cuda()
    x, w = latgen.random_sources(dims, 2, 6)
    dx, dw = to_dev(x), to_dev(w)
    xp, wp, t1, t2, back = (torch.empty_like(dx) for _ in range(5))
    b.nk_spinor_pack_device(lat.h, dx, xp)
    b.nk_spinor_pack_device(lat.h, dw, wp)
    b.nk_spinor_unpack_device(lat.h, xp, back)
    torch.cuda.synchronize()
    assert torch.equal(back, dx)
    assert abs(torch.vdot(wp, xp).item() - torch.vdot(dw, dx).item()) < 1e-12 * abs(torch.vdot(dw, dx).item())
    # one application: packed == canonical, bit for bit
    ref1 = torch.empty_like(dx)
    b.nk_apply_dw_device(lat.h, M_W, mu, True, dx, ref1)
    b.nk_apply_dw_packed_device(lat.h, M_W, mu, True, xp, t1)
    b.nk_spinor_unpack_device(lat.h, t1, back)
    torch.cuda.synchronize()
    assert torch.equal(back, ref1)
    # the fused pair: packed == canonical
    av, adw, avp, adwp = (torch.empty_like(dx) for _ in range(4))
    b.nk_apply_pair_device(lat.h, M_W, mu, dx, dw, av, adw)
    b.nk_apply_pair_packed_device(lat.h, M_W, mu, xp, wp, avp, adwp)
    b.nk_spinor_unpack_device(lat.h, avp, back)
    torch.cuda.synchronize()
    assert torch.equal(back, av)
    b.nk_spinor_unpack_device(lat.h, adwp, back)
    torch.cuda.synchronize()
    assert torch.equal(back, adw)
    # two applications without leaving the packed layout, against the oracle
    b.nk_apply_dw_packed_device(lat.h, M_W, mu, True, t1, t2)
    b.nk_spinor_unpack_device(lat.h, t2, back)
    torch.cuda.synchronize()
    got = to_host(back).reshape(x.shape)
    ref = W.dw_apply(u, W.dw_apply(u, x, M_W, mu, g5=True), M_W, mu, g5=True)
    assert rel(got, ref) < TOL * 20
    lat.close()


def test_packed_entry_points_reject_aliasing():
    """argument checks on the host, before any launch"""
    b = nk()
    torch = torch_cuda()
    dims = (2, 2, 2, 2)
    lat, _ = make_lattice(dims, 0.5, seed=1)
    a = torch.zeros(12 * 16, dtype=torch.complex128, device="cuda")
    c = torch.zeros_like(a)
    for call in (lambda: b.nk_apply_dw_packed_device(lat.h, M_W, 0.0, True, a, a),
                 lambda: b.nk_apply_pair_packed_device(lat.h, M_W, 0.0, a, c, a, c),
                 lambda: b.nk_apply_pair_packed_device(lat.h, M_W, 0.0, a, c, c, c),
                 lambda: b.nk_spinor_pack_device(lat.h, a, a),
                 lambda: b.nk_spinor_unpack_device(lat.h, a, a, nrhs=0)):
        with pytest.raises(b.NKError) as ei:
            call()
        assert ei.value.code == b.NK_EINVAL
    lat.close()
