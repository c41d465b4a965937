"""Pins of the learned Roberts-Higham scaling oracle (oracle/learned.py)."""
import numpy as np
import pytest

import latgen
from oracle import learned as L
from oracle import rh as orh


def _rand_matrix(n, seed, shift=3.0, hermitian=False):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if hermitian:
        a = a + a.conj().T
    return a + shift * np.diag(np.where(np.arange(n) % 3 == 0, -1.0, 1.0))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spectral_loss_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    lam = np.linalg.eigvals(_rand_matrix(30, seed))
    y = 0.4 * rng.standard_normal(L.T)
    _, g = L.spectral_loss(lam, y)
    h = 1e-6
    fd = np.array([(L.spectral_loss(lam, y + h * e)[0] - L.spectral_loss(lam, y - h * e)[0]) / (2 * h)
                   for e in np.eye(L.T)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_spectral_loss_gradient_real_spectrum():
    lam = np.linalg.eigvalsh(_rand_matrix(25, 5, hermitian=True)).astype(np.complex128)
    y = np.array([0.3, -0.2, 0.1, 0.05])
    _, g = L.spectral_loss(lam, y)
    h = 1e-6
    fd = np.array([(L.spectral_loss(lam, y + h * e)[0] - L.spectral_loss(lam, y - h * e)[0]) / (2 * h)
                   for e in np.eye(L.T)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    p = latgen.mlp_init(4).astype(np.float64)
    p[L.NTRAIN:L.NTRAIN + L.NIN] = rng.standard_normal(L.NIN) * 0.1
    p[L.NTRAIN + L.NIN:] = 1.0 + 0.2 * rng.random(L.NIN)
    p[:L.NTRAIN] += 0.05 * rng.standard_normal(L.NTRAIN)  # non-zero biases
    f = rng.standard_normal((5, L.NIN))
    dy = rng.standard_normal((5, L.T))
    y, acts = L.forward(p, f)
    g = L.backward(p, acts, dy)
    idx = rng.choice(L.NTRAIN, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (np.sum(dy * L.forward(p + e, f)[0]) - np.sum(dy * L.forward(p - e, f)[0])) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_eigenvalue_model_matches_dense_scaled_iteration():
    """The loss's premise: T dense Roberts-Higham steps with
    mu_t = |det S_t|^{-1/n} exp(y_t) move every eigenvalue by the scalar map
    (S_T = r(S_0) for a rational r, and log|det S_t| = sum log|z_t|)."""
    s0 = _rand_matrix(24, 7, shift=2.0)
    y = np.array([-0.7, 0.2, -0.1, 0.05])
    st, it, _ = orh.roberts_higham(s0, tol=0.0, maxit=L.T,
                                   scale=lambda k, s: orh.determinant_scale(k, s) * float(np.exp(y[k])))
    assert it == L.T
    lam = np.linalg.eigvals(s0)
    zt = L.scaled_orbit(lam, y)[0][-1]
    got = np.linalg.eigvals(st)
    # match each predicted eigenvalue to its nearest computed one
    err = max(np.min(np.abs(got - z)) for z in zt)
    assert err < 1e-8 * np.max(np.abs(zt))


def test_determinant_scaled_orbit_of_two_eigenvalues():
    """Spectrum {a, b} > 0 with y = 0: mu_0 = 1/sqrt(ab) sends both to
    (a + b) / (2 sqrt(ab)), and mu_1 = 1 / that value sends both to 1."""
    a, b = 0.3, 12.0
    z, lmu = L.scaled_orbit(np.array([a, b], np.complex128), np.zeros(L.T))
    assert abs(lmu[0] + 0.5 * np.log(a * b)) < 1e-14
    z1 = (a + b) / (2 * np.sqrt(a * b))
    assert np.allclose(z[1], z1, rtol=1e-14)
    assert np.allclose(z[2], 1.0, rtol=1e-14)


def test_determinant_scaling_reaches_the_sign_of_one_eigenvalue_in_one_step():
    """A single eigenvalue z: mu_0 = 1/|z| maps a real z to exactly sgn(z),
    so the loss is at its floor log(FLOOR) / 2 and its gradient vanishes."""
    for lam in (5.0, -0.2):
        loss, g = L.spectral_loss(np.array([lam + 0j]), np.zeros(L.T))
        assert abs(loss - 0.5 * np.log(L.FLOOR)) < 1e-12
        assert np.all(np.abs(g) < 1e-6)


def test_scaling_never_changes_the_limit():
    s0 = _rand_matrix(16, 11, shift=2.5)
    ref, _, _ = orh.roberts_higham(s0)
    for y in (np.array([1.0, -0.5, 0.3, 0.0]), np.array([-2.0, 0.0, 0.0, 0.0])):
        sc = lambda k, s, yy=y: orh.determinant_scale(k, s) * float(np.exp(yy[k])) if k < L.T else None
        got, _, _ = orh.roberts_higham(s0, scale=sc)
        assert np.linalg.norm(got - ref) < 1e-10 * np.linalg.norm(ref)


def test_features_scale_and_permutation_invariance():
    s = _rand_matrix(18, 2)
    f = L.features(s)
    f2 = L.features(3.7 * s)
    assert abs(f2[1] - f[1] - np.log(3.7)) < 1e-12
    keep = [i for i in range(L.NIN) if i != 1]
    assert np.allclose(f[keep], f2[keep], atol=1e-12)
    perm = np.random.default_rng(0).permutation(18)
    f3 = L.features(s[np.ix_(perm, perm)])
    assert np.allclose(f, f3, atol=1e-12)


def test_features_of_a_diagonal_matrix():
    d = np.array([2.0, -1.0, 0.5, 4.0])
    f = L.features(np.diag(d).astype(np.complex128))
    rms = np.sqrt(np.mean(d ** 2))
    assert abs(f[0] - np.log(4)) < 1e-14
    assert abs(f[1] - np.log(rms)) < 1e-14
    assert abs(f[4] - d.sum() / (4 * rms)) < 1e-14
    assert abs(f[9] - 0.75) < 1e-14          # three positive diagonal entries
    assert f[12] == -50.0 and f[13] == -50.0  # Hermitian, no off-diagonal part (clamped logs)
    assert f[15] == 0.0                       # no Gershgorin disc crosses the imaginary axis


def test_adam_first_step_is_lr_times_sign():
    p = np.zeros(L.NPARAMS)
    g = np.zeros(L.NTRAIN)
    g[:5] = [3.0, -2.0, 1e-3, -1e-2, 0.5]
    m = np.zeros(L.NTRAIN)
    v = np.zeros(L.NTRAIN)
    L.adam_step(p, g, m, v, 1, 0.01)
    assert np.allclose(p[:5], -0.01 * np.sign(g[:5]), rtol=1e-4)
    assert np.all(p[5:] == 0)


def _backward_fd_error(backward):
    rng = np.random.default_rng(9)
    p = latgen.mlp_init(1).astype(np.float64)
    p[:L.NTRAIN] += 0.2 * rng.standard_normal(L.NTRAIN)
    f = rng.standard_normal((3, L.NIN))
    dy = rng.standard_normal((3, L.T))
    _, acts = L.forward(p, f)
    g = backward(p, acts, dy)
    h, err = 1e-6, 0.0
    for i in rng.choice(L.NTRAIN, 60, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (np.sum(dy * L.forward(p + e, f)[0]) - np.sum(dy * L.forward(p - e, f)[0])) / (2 * h)
        err = max(err, abs(fd - g[i]) / max(1.0, abs(fd)))
    return err


def test_planted_mistake_in_backward_is_caught():
    """A dropped tanh derivative in the last hidden layer, planted in a copy
    of the oracle's backward pass, fails the finite-difference pin."""
    def planted(p, acts, dy):
        x, a1, a2, a3 = acts
        w = L.unpack(p)
        dy = np.atleast_2d(dy)
        g = {"W4": dy.T @ a3, "b4": dy.sum(0)}
        d3 = dy @ w["W4"]  # mistake: no (1 - a3^2)
        g["W3"], g["b3"] = d3.T @ a2, d3.sum(0)
        d2 = (d3 @ w["W3"]) * (1.0 - a2 * a2)
        g["W2"], g["b2"] = d2.T @ a1, d2.sum(0)
        d1 = (d2 @ w["W2"]) * (1.0 - a1 * a1)
        g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
        return np.concatenate([g[n].reshape(-1) for n in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])
    assert _backward_fd_error(L.backward) < 1e-6
    assert _backward_fd_error(planted) > 1e-3


def _loss_grad_planted(lam, y, drop_conj=False, drop_det=False):
    """A copy of the oracle's loss gradient with one planted mistake."""
    n = lam.size
    z, lmu = L.scaled_orbit(lam, y)
    sg = np.where(lam.real > 0, 1.0, -1.0)
    e = np.abs(z[-1] - sg) ** 2
    d = 0.5 * np.log(e + L.FLOOR)
    ex = np.exp(L.KAPPA * (d - d.max()))
    gz = ex / ex.sum() * (z[-1] - sg) / (e + L.FLOOR)
    grad = np.zeros(len(y))
    for t in range(len(y) - 1, -1, -1):
        mu = np.exp(lmu[t])
        wv = mu * z[t]
        fp = 0.5 * (1.0 - 1.0 / (wv * wv))
        gw = (fp if drop_conj else np.conj(fp)) * gz
        glm = np.sum((np.conj(gw) * wv).real)
        grad[t] = glm
        gz = mu * gw - (0.0 if drop_det else glm * z[t] / (n * np.abs(z[t]) ** 2))
    return grad


@pytest.mark.parametrize("mistake", ["drop_conj", "drop_det"])
def test_planted_mistake_in_loss_gradient_is_caught(mistake):
    """Dropping the conjugate in the chain rule through z -> (w + 1/w) / 2, or
    the path through the determinant scale, fails the finite-difference pin
    on a complex spectrum."""
    lam = np.linalg.eigvals(_rand_matrix(20, 4))
    y = np.array([0.2, -0.3, 0.1, 0.0])
    h = 1e-6
    fd = np.array([(L.spectral_loss(lam, y + h * e)[0] - L.spectral_loss(lam, y - h * e)[0]) / (2 * h)
                   for e in np.eye(L.T)])
    assert np.allclose(L.spectral_loss(lam, y)[1], fd, rtol=1e-6, atol=1e-8)
    assert np.allclose(_loss_grad_planted(lam, y), fd, rtol=1e-6, atol=1e-8)  # the copy itself is right
    assert not np.allclose(_loss_grad_planted(lam, y, **{mistake: True}), fd, rtol=1e-3, atol=1e-5)
