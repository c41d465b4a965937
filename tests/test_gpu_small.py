"""GPU parity of the small problem: Roberts-Higham (Eq. (4)) and the nested
projection (Sec. 3, Eqs. (5)-(6)).

* nk_rh_sign against the oracle's RH and the spectral sign, for single and
  batched matrices of uneven sizes (several 64 x 64 update tiles and ragged
  panel tails), complex and real symmetric.
* nk_small_sign against oracle.nested.small_sign on Ritz matrices H_k built by
  the oracle (non-nested l = 0 and nested l > 0, Hermitian and not).
Tolerances: the results are sign functions of moderately conditioned
matrices; both sides are FP64 with different (but both pivoted) eliminations,
so they agree to ~cond * 1e-16.  1e-10 relative is used.
"""
import numpy as np
import pytest

import latgen
from oracle import dense as D
from oracle import nested as N
from oracle import rh as R
from oracle import wilson as W
from tests.gpu_helpers import M_W, banner, nk, rel

pytestmark = pytest.mark.gpu


def _rand_matrix(n, seed, herm=False):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if herm:
        a = a + a.conj().T
    a += 0.5 * np.diag(np.sign(rng.standard_normal(n)))
    return a


@pytest.mark.parametrize("n", [1, 7, 16, 17, 64, 130, 301, 500, 1000])
def test_rh_single_matches_oracle(n):
    banner(f"rh single n={n}")
    b = nk()
    a = _rand_matrix(n, n)
    s, it, rc = b.nk_rh_sign(a)
    so, ito, _ = R.roberts_higham(a)
    assert rel(s[0], so) < 1e-10
    assert rel(s[0], D.sign_spectral(a, hermitian=False)) < 1e-9
    assert abs(int(it[0]) - ito) <= 1


@pytest.mark.parametrize("n", [200, 500])
def test_rh_newton_schulz_tail_same_limit(n):
    """The Newton-Schulz tail (orders > 128) reaches the limit of the
    inversion-only iteration (Eq. (4)) and the oracle's, in about as many
    steps (both converge quadratically)."""
    banner(f"rh newton-schulz tail n={n}")
    b = nk()
    a = _rand_matrix(n, 7 * n)
    old = b.nk_rh_newton_schulz(False)
    try:
        s0, it0, _ = b.nk_rh_sign(a)
        b.nk_rh_newton_schulz(True)
        s1, it1, _ = b.nk_rh_sign(a)
    finally:
        b.nk_rh_newton_schulz(old)
    so, ito, _ = R.roberts_higham(a)
    print(f"[rh] n={n}: iterations inversion-only {it0[0]}, with the tail {it1[0]}, oracle {ito}; "
          f"tail vs inversion-only {rel(s1[0], s0[0]):.2e}", flush=True)
    assert rel(s0[0], so) < 1e-10 and rel(s1[0], so) < 1e-10
    assert rel(s1[0], s0[0]) < 1e-11
    assert abs(int(it1[0]) - int(it0[0])) <= 1


def test_rh_batched_uneven_sizes():
    banner("rh batched, uneven sizes")
    b = nk()
    sizes = [40, 300, 129, 64, 1, 250]
    ld = max(sizes)
    S = np.zeros((len(sizes), ld, ld), np.complex128)
    mats = []
    for i, n in enumerate(sizes):
        a = _rand_matrix(n, 100 + i, herm=(i % 2 == 0))
        mats.append(a)
        S[i, :n, :n] = a
    out, it, rc = b.nk_rh_sign(S, n=sizes)
    for i, n in enumerate(sizes):
        so, ito, _ = R.roberts_higham(mats[i])
        assert rel(out[i, :n, :n], so) < 1e-10, i
        assert abs(int(it[i]) - ito) <= 1


def test_rh_det_scaling_same_limit():
    banner("rh determinant scaling")
    b = nk()
    a = _rand_matrix(90, 5)
    s0, it0, _ = b.nk_rh_sign(a)
    s1, it1, _ = b.nk_rh_sign(a, scaling=b.NK_RH_DET)
    assert rel(s1[0], s0[0]) < 1e-10
    assert it1[0] <= it0[0]
    so, _, _ = R.roberts_higham(a, scale=R.determinant_scale)
    assert rel(s1[0], so) < 1e-10


@pytest.fixture(scope="module", params=[0.0, 0.3])
def ritz(request):
    mu = request.param
    dims = (4, 4, 4, 4)
    u = latgen.random_gauge(dims, 0.6, 0)
    x = latgen.random_sources(dims, 1, 0)[0]
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, mu).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -mu).reshape(-1)
    kr = N.outer_basis(f, fd, x.reshape(-1), 150, mu == 0.0)
    return mu, kr.H


@pytest.mark.parametrize("ell", [0, 1, 20, 45, 150])
def test_small_sign_matches_oracle(ritz, ell):
    mu, H = ritz
    herm = mu == 0.0
    banner(f"small_sign k={H.k} ell={ell} mu={mu}")
    b = nk()
    z, info, rc = b.nk_small_sign(H.k, ell, herm, H.alpha, H.beta, H.delta)
    zo, io = N.small_sign(H, ell, herm)
    assert rel(z, zo) < 1e-10
    assert info.ell_used == (min(ell, H.k) if ell else 0)
    assert abs(info.rh_iters - io["rh_iters"]) <= 1
    assert info.rh_residual < 1e-9


@pytest.mark.parametrize("k", [100, 150])
@pytest.mark.parametrize("maxit", [2, 3, 100])
def test_rh_residual_is_s_squared_minus_one(ritz, k, maxit):
    """info.rh_residual is |S^2 - I|_F / sqrt(n) of the final Roberts-Higham
    iterate: against the oracle's iterate after the same number of steps on
    the plain form's H_k (k = 100 runs the one-workgroup kernel, 150 the
    blocked inverse), unconverged (2, 3 steps: residual of order one) and
    converged (below 1e-9)."""
    mu, H = ritz
    herm = mu == 0.0
    b = nk()
    p = b.nk_sign_params_default(rh_maxit=maxit)
    z, info, rc = b.nk_small_sign(k, 0, herm, H.alpha[:k], H.beta[:k], H.delta[:k], p)
    hk = H.dense()[:k, :k]
    S, it, _ = R.roberts_higham(hk, maxit=maxit)
    ref = np.linalg.norm(S @ S - np.eye(k)) / np.sqrt(k)
    print(f"k={k} maxit={maxit}: GPU {info.rh_residual:.6e} oracle {ref:.6e} ({info.rh_iters} / {it} steps)", flush=True)
    assert info.rh_iters == it
    if maxit < 100:
        assert rc == b.NK_WARN_NOTCONV
        assert abs(info.rh_residual - ref) <= 1e-8 * ref
    else:
        assert info.rh_residual < 1e-9 and ref < 1e-9


@pytest.mark.parametrize("ell", [1, 20, 45, 150])
def test_small_sign_arnoldi_matches_oracle(ritz, ell):
    """The Arnoldi inner option against the oracle's Arnoldi (Hessenberg H_l),
    and at mu = 0, where B is Hermitian, against the Lanczos inner space."""
    mu, H = ritz
    herm = mu == 0.0
    banner(f"small_sign arnoldi k={H.k} ell={ell} mu={mu}")
    b = nk()
    p = b.nk_sign_params_default(inner=b.NK_INNER_ARNOLDI)
    z, info, rc = b.nk_small_sign(H.k, ell, herm, H.alpha, H.beta, H.delta, p)
    zo, io = N.small_sign(H, ell, herm, inner="arnoldi")
    assert rel(z, zo) < 1e-10
    assert info.ell_used == min(ell, H.k)
    if herm:
        zs, _, _ = b.nk_small_sign(H.k, ell, herm, H.alpha, H.beta, H.delta)
        assert rel(z, zs) < 1e-10


def test_small_sign_ragged_k(ritz):
    mu, H = ritz
    herm = mu == 0.0
    b = nk()
    for k in (2, 3, 65, 97):
        Hk = H.leading(k)
        z, info, rc = b.nk_small_sign(k, k // 2, herm, Hk.alpha, Hk.beta, Hk.delta)
        zo, _ = N.small_sign(Hk, k // 2, herm)
        assert rel(z, zo) < 1e-10, k


# every launch shape of the blocked inverse that covers each order: (rows per
# thread, panel threads), each with update tiles 32 and 64
_SHAPES_LE_512 = [(1, 512), (1, 1024), (2, 256), (2, 512)]
_SHAPES_LE_2048 = [(2, 1024), (4, 512)]


@pytest.mark.parametrize("sizes, shapes", [([300, 150, 229, 1], _SHAPES_LE_512),
                                           ([1100, 700], _SHAPES_LE_2048)])
def test_rh_every_launch_shape_gives_the_same_bits(sizes, shapes):
    """The autotuner's choices (panel threads, rows per thread, update tile)
    change no arithmetic: every shape returns the same bits, which match the
    oracle's Roberts-Higham iteration."""
    banner(f"rh launch shapes, sizes {sizes}")
    b = nk()
    ld = max(sizes)
    S = np.zeros((len(sizes), ld, ld), np.complex128)
    mats = []
    for i, n in enumerate(sizes):
        a = _rand_matrix(n, 300 + i, herm=(i % 2 == 1))
        mats.append(a)
        S[i, :n, :n] = a
    ref = None
    try:
        for rm, pth in shapes:
            for tile in (32, 64):
                b.nk_rh_tile_force(rm, pth, tile)
                out, it, rc = b.nk_rh_sign(S, n=sizes)
                if ref is None:
                    ref = (out, it)
                    for i, n in enumerate(sizes):
                        so, ito, _ = R.roberts_higham(mats[i])
                        assert rel(out[i, :n, :n], so) < 1e-10, i
                        assert abs(int(it[i]) - ito) <= 1
                else:
                    assert np.array_equal(out, ref[0]), (rm, pth, tile)
                    assert np.array_equal(it, ref[1]), (rm, pth, tile)
    finally:
        b.nk_rh_tile_force(0, 0, 0)
    # back to the autotuner: it picks a shape for this class, same bits again
    out, it, _ = b.nk_rh_sign(S, n=sizes)
    assert np.array_equal(out, ref[0])
    choice = b.nk_rh_tile_choice(ld, len(sizes))
    assert choice is not None and choice[2] * choice[1] >= ld, choice
