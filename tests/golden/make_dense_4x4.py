"""Write tests/golden/dense_4x4.npz: sgn(A) b by the spectral definition
(Eq. fAdef: dense eigendecomposition, sgn of the real parts) on the 4^4
lattice (SU(3) links eps = 0.5, seed 4401, m0 = 1.6, Gaussian source seed
4402) at mu = 0 (Hermitian, eigh) and mu = 0.3 (eig), together with the
oracle's nested method at (k, ell) = (800, 160) and (1000, 200) and its
distance to the dense result, the pin that the GPU tests at 1e-10 rely on.

Calls only ``oracle`` and ``nks_inputs``.  Minutes (the two 3072 x 3072
eigendecompositions).
Usage: python tests/golden/make_dense_4x4.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import nks_inputs as I  # noqa: E402
from oracle import dirac, nested  # noqa: E402

DIMS, EPS, SEED, SRC, M0 = (4, 4, 4, 4), 0.5, 4401, 4402, 1.6
CASES = ((0.0, 800, 160), (0.3, 1000, 200))


def main():
    b = I.gaussian_source(DIMS, SRC)
    out = {}
    for mu, k, ell in CASES:
        t = time.time()
        op = dirac.Operator(I.su3_links(DIMS, EPS, SEED), DIMS, M0, mu)
        y = nested.sign_exact_dense(op, b).ravel()
        y_k, _ = nested.sign_apply(op, b, k, ell)
        e = nested.rel_err(y_k, y)
        tag = f"mu{mu:g}"
        out[f"y_{tag}"] = y
        out[f"k_{tag}"] = k
        out[f"ell_{tag}"] = ell
        out[f"oracle_err_{tag}"] = e
        print(f"mu={mu}: oracle nested k={k} ell={ell} vs dense {e:.2e} ({time.time() - t:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "dense_4x4.npz"), **out)


if __name__ == "__main__":
    main()
