"""Shared helpers of the GPU tests: inputs from latgen, the C ABI through the binding."""
from __future__ import annotations

import numpy as np

import latgen

M_W = -1.0


def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch


def nk():
    from paper_0910_2918_amd import nk as _nk

    _nk.library()  # fail loudly when the HIP library is not built
    return _nk


def make_lattice(dims, eps, seed=0, unit=False):
    b = nk()
    lat = b.Lattice(dims)
    u = latgen.unit_gauge(dims) if unit else latgen.random_gauge(dims, eps, seed)
    b.nk_gauge_set(lat.h, u)
    return lat, u


def to_dev(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)).to("cuda")


def to_host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def rel(a, b) -> float:
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)


def perturbed(x: np.ndarray, seed: int = 99, size: float = 1e-15) -> np.ndarray:
    """x with every entry changed by a relative amount of about `size`
    (complex Gaussian, seeded): a change at the level of FP64 rounding."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    return x * (1.0 + size * d)


def method_bound(sens: float) -> float:
    """Method-level tolerance of GPU against oracle at the same (k, l): the
    oracle's own result moves by `sens` when its source changes at the
    rounding level (perturbed), and the GPU, whose reductions round
    differently at every step of the recurrence, may differ by up to 10
    times that (measured: at most 3 times, over every method-level case),
    and by no more than 1e-12 where the recurrence amplifies nothing."""
    return max(1e-12, 10.0 * sens)
