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
