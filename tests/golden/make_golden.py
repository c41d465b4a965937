"""Write the stored expected values used by the tests.

Calls only the CPU oracle (and the seeded input generators); nothing here
touches the HIP library.  Each file is the exact sign sgn(gamma5 Dw(mu)) x of
the spectral definition (Eq. (2), with sgn(z) = sgn(Re z)) on the 4^4
workload: m_w = -1, link width eps = 0.4, gauge seed 0, source seed 0.

Usage: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import latgen  # noqa: E402
from oracle import dense, wilson  # noqa: E402

DIMS = (4, 4, 4, 4)


def main():
    u = latgen.random_gauge(DIMS, 0.4, 0)
    x = latgen.random_sources(DIMS, 1, 0)[0].reshape(-1)
    for mu, name in ((0.0, "sign_4x4x4x4_mu0_eps0.4.npy"), (0.3, "sign_4x4x4x4_mu0.3_eps0.4.npy")):
        a = wilson.dense_matrix(u, -1.0, mu)
        y = dense.sign_spectral(a, hermitian=(mu == 0.0)) @ x
        np.save(os.path.join(HERE, name), y)
        print(name, "min|Re lambda| =", dense.min_abs_re_eig(a))


if __name__ == "__main__":
    main()
