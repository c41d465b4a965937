"""Learned scaling of the Roberts-Higham iteration (an extension of Eq. (4)).

The scaled iteration S_{n+1} = (mu_n S_n + (mu_n S_n)^{-1}) / 2 with any
mu_n > 0 has the same limit sgn(S_0): the scalar argument of Eq. (7)
(sgn Re(z + 1/z) = sgn Re z) holds for mu z as well.  The factors therefore
change only how many iterations are needed.  Here the factor of each of the
first T steps is determinant scaling times a learned correction,

    mu_t = |det S_t|^{-1/n} exp(y_t),

with y_0 .. y_{T-1} predicted by a small network from 16 cheap features f
of S_0 = H_ell:

    x  = (f - mean) * inv_std                      (16)
    a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), a3 = tanh(W3 a2 + b3)   (64 each)
    y  = W4 a3 + b4                                                      (T)

so y = 0 is plain determinant scaling.  Training needs no labels: for a
diagonalisable S_0 every eigenvalue follows the scalar map
z <- (mu z + 1/(mu z)) / 2, and log|det S_t| = sum_i log|z_{i,t}|, so the
distance d_i = log|z_{i,T} - sgn Re lambda_i| after T steps follows from the
spectrum alone; the loss is the smooth maximum
L = (1/kappa) log(mean_i exp(kappa d_i)) with d_i = log(|z_{i,T} - sgn|^2 + FLOOR) / 2.
FLOOR = 1e-14 makes every distance below 1e-7 count as converged: quadratic
convergence takes such an eigenvalue to 1e-14 in one more step, so a schedule
gains nothing by going further, and without the floor the loss has sharp
valleys (log 0 at exact hits) whose gradients swamp everything else.

Everything here is plain FP64 numpy written from these definitions: the
features, the forward pass, the loss and its gradient by the chain rule,
the backward pass and an Adam step.  It is pinned by central finite
differences (gradients), by the dense oracle Roberts-Higham iteration run
with the same factors (the eigenvalue model), and by closed forms.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

NIN, NH, T = 16, 64, 4
KAPPA = 4.0
TINY = 1e-30  # guards logs of features
FLOOR = 1e-14  # squared distance below which an eigenvalue counts as converged

# flat parameter layout: trainable part, then the feature standardisation
_SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NH)), ("b3", (NH,)),
           ("W4", (T, NH)), ("b4", (T,))]
NTRAIN = sum(int(np.prod(s)) for _, s in _SHAPES)
NPARAMS = NTRAIN + 2 * NIN


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in _SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    out["mean"] = np.asarray(p[o:o + NIN], dtype=np.float64)
    out["istd"] = np.asarray(p[o + NIN:o + 2 * NIN], dtype=np.float64)
    return out


def pack(d: dict) -> np.ndarray:
    parts = [np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in _SHAPES]
    parts += [np.asarray(d["mean"], np.float64), np.asarray(d["istd"], np.float64)]
    return np.concatenate(parts)


def clampf(v: float) -> float:
    return float(min(50.0, max(-50.0, v)))


def features(s: np.ndarray) -> np.ndarray:
    """16 features of a dense complex n x n matrix, O(n^2) work."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    a = np.abs(s)
    fro = np.sqrt(np.sum(a * a))
    rms = fro / np.sqrt(n)
    lr = np.log(rms + TINY)
    d = np.diag(s)
    ad = np.abs(d)
    rad = a.sum(axis=1) - ad  # Gershgorin radii
    offd = np.sqrt(max(fro * fro - np.sum(ad * ad), 0.0))
    herm = np.linalg.norm(s - s.conj().T)
    logd = np.log(ad + TINY)
    f = np.array([
        np.log(n),
        lr,
        np.log(a.sum(axis=1).max() + TINY) - lr,
        np.log(a.sum(axis=0).max() + TINY) - lr,
        d.real.sum() / (n * (rms + TINY)),
        d.imag.sum() / (n * (rms + TINY)),
        np.log(ad.max() + TINY) - lr,
        np.log(ad.min() + TINY) - lr,
        np.log(np.abs(d.real).min() + TINY) - lr,
        np.mean(d.real > 0),
        logd.mean() - lr,
        logd.std(),
        np.log(herm / (fro + TINY) + TINY),
        np.log(offd / (np.sqrt(np.sum(ad * ad)) + TINY) + TINY),
        np.log(rad.max() + TINY) - lr,
        np.mean(np.abs(d.real) < rad),
    ])
    return np.array([clampf(v) for v in f])


def forward(p: np.ndarray, f: np.ndarray):
    """y (B x T) for features f (B x 16); also the activations for backward."""
    w = unpack(p)
    f = np.atleast_2d(np.asarray(f, np.float64))
    x = (f - w["mean"]) * w["istd"]
    a1 = np.tanh(x @ w["W1"].T + w["b1"])
    a2 = np.tanh(a1 @ w["W2"].T + w["b2"])
    a3 = np.tanh(a2 @ w["W3"].T + w["b3"])
    y = a3 @ w["W4"].T + w["b4"]
    return y, (x, a1, a2, a3)


def backward(p: np.ndarray, acts, dy: np.ndarray) -> np.ndarray:
    """Gradient of sum_b <dy_b, y_b> with respect to the trainable parameters
    (flat, NTRAIN entries; the standardisation is not trained)."""
    w = unpack(p)
    x, a1, a2, a3 = acts
    dy = np.atleast_2d(dy)
    g = {"W4": dy.T @ a3, "b4": dy.sum(0)}
    d3 = (dy @ w["W4"]) * (1.0 - a3 * a3)
    g["W3"], g["b3"] = d3.T @ a2, d3.sum(0)
    d2 = (d3 @ w["W3"]) * (1.0 - a2 * a2)
    g["W2"], g["b2"] = d2.T @ a1, d2.sum(0)
    d1 = (d2 @ w["W2"]) * (1.0 - a1 * a1)
    g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
    return np.concatenate([g[name].reshape(-1) for name, _ in _SHAPES])


def log_det_scale(z: np.ndarray) -> float:
    """log of the determinant scale |det S|^{-1/n} from the eigenvalues z."""
    return float(-np.mean(np.log(np.abs(z))))


def scaled_orbit(lam: np.ndarray, y: np.ndarray):
    """z_t (t = 0..T, one row per step) and log mu_t of the scaled scalar map
    with mu_t = |det S_t|^{-1/n} exp(y_t)."""
    z = [np.asarray(lam, np.complex128)]
    lmu = []
    for t in range(len(y)):
        lm = log_det_scale(z[-1]) + y[t]
        wv = np.exp(lm) * z[-1]
        z.append(0.5 * (wv + 1.0 / wv))
        lmu.append(lm)
    return np.array(z), np.array(lmu)


def spectral_loss(lam: np.ndarray, y: np.ndarray):
    """(L, dL/dy) for one matrix with eigenvalues lam."""
    lam = np.asarray(lam, np.complex128)
    y = np.asarray(y, np.float64)
    n = lam.size
    z, lmu = scaled_orbit(lam, y)
    sg = np.where(lam.real > 0, 1.0, -1.0)
    e = np.abs(z[-1] - sg) ** 2
    dlog = 0.5 * np.log(e + FLOOR)
    m = dlog.max()
    ex = np.exp(KAPPA * (dlog - m))
    loss = m + np.log(ex.sum() / n) / KAPPA
    wgt = ex / ex.sum()  # dL/dd_i
    # gradients as complex numbers dRe + i dIm
    gz = wgt * (z[-1] - sg) / (e + FLOOR)
    grad = np.zeros(len(y))
    for t in range(len(y) - 1, -1, -1):
        mu = np.exp(lmu[t])
        wv = mu * z[t]
        gw = np.conj(0.5 * (1.0 - 1.0 / (wv * wv))) * gz  # through z_{t+1} = (w + 1/w) / 2
        glm = np.sum((np.conj(gw) * wv).real)               # dL/dlog mu_t (w = mu z_t)
        grad[t] = glm                                       # log mu_t = y_t + log det scale(z_t)
        # through w = mu z_t directly, and through the determinant scale:
        # d(-mean log|z_i|)/dz_i = -(1/n) z_i / |z_i|^2
        gz = mu * gw - glm * z[t] / (n * np.abs(z[t]) ** 2)
    return float(loss), grad


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update of the trainable part of p (in place); t counts from 1."""
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[:NTRAIN] -= lr * mh / (np.sqrt(vh) + eps)
    return p
