"""Write the Ritz matrix H_k of the benchmark workload, computed by the oracle.

16^4 lattice, mu = 0.3, m_w = -1, link width 0.8, gauge seed 0, source seed 0
(the benchmark's own inputs), k = 500 steps of the oracle's two-sided Lanczos
(Sec. 2): the diagonal alpha, super-diagonal beta and sub-diagonal delta of
H_k, about 24 KB.  Calls only the oracle and the seeded input generators;
the run takes 5-15 minutes of host time.  bench.py times the oracle's small
problem on this H_k, and the GPU tests compare the library's first outer
coefficients with it.

Usage: python tests/golden/make_hk.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import latgen  # noqa: E402
from oracle import krylov, wilson  # noqa: E402

DIMS, MU, EPS, K = (16, 16, 16, 16), 0.3, 0.8, 500
NAME = "hk_16x16x16x16_mu0.3_eps0.8_k500.npz"


def main():
    u = latgen.random_gauge(DIMS, EPS, 0)
    x = latgen.random_sources(DIMS, 1, 0)[0]
    f = lambda v: wilson.a_apply(u, v.reshape(x.shape), -1.0, MU).reshape(-1)
    fd = lambda v: wilson.a_apply(u, v.reshape(x.shape), -1.0, -MU).reshape(-1)
    t0 = time.time()
    kr = krylov.two_sided_lanczos(f, fd, x.reshape(-1), K)
    h = kr.H
    np.savez(os.path.join(HERE, NAME), alpha=h.alpha, beta=h.beta, delta=h.delta)
    print(f"{NAME}: k = {h.k}, breakdown = {kr.breakdown}, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
