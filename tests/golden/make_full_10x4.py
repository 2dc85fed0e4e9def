"""Write tests/golden/point4_full_10x4.npz: the oracle's converged sgn(A) b as
complete vectors for four of the benchmark's point sources on the 10^4
lattice (eps = 0.35, link seed 10401, m0 = 1.6): (spin, colour) = (0, 0) and
(2, 1) at mu = 0, (0, 0) and (3, 2) at mu = 0.2.  Same reference as
point12_10x4.json (make_point12_10x4.py): the non-nested Krylov-Ritz result
with the spectral sign of H_k at k = 1400 (mu = 0) and 1000 (mu = 0.2), and
its change from k = 1200 / 800 as its accuracy.

Calls only ``oracle`` and ``nks_inputs``.  A few minutes on 4 cores.
Usage: python tests/golden/make_full_10x4.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)
os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")

import nks_inputs as I  # noqa: E402
from make_point12_10x4 import DIMS, K_CHECK, K_REF, sign_e1  # noqa: E402
from oracle import dirac, krylov  # noqa: E402

SOURCES = ((0.0, 0, 0), (0.0, 2, 1), (0.2, 0, 0), (0.2, 3, 2))


def main():
    links = I.su3_links(DIMS, 0.35, 10401)
    ys, changes = [], []
    for mu, spin, colour in SOURCES:
        t = time.time()
        op = dirac.Operator(links, DIMS, 1.6, mu)
        b = I.point_source(DIMS, spin, colour).ravel()
        if mu == 0.0:
            kr = krylov.lanczos(op.matvec, b, K_REF[mu])
        else:
            kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, K_REF[mu])
        y = kr.bnorm * (kr.V @ sign_e1(kr.alpha, kr.beta, kr.gamma, mu == 0.0))
        kc = min(K_CHECK[mu], kr.k_used)
        y2 = kr.bnorm * (kr.V[:, :kc] @ sign_e1(kr.alpha[:kc], kr.beta[:kc - 1], kr.gamma[:kc - 1], mu == 0.0))
        ch = float(np.linalg.norm(y - y2) / np.linalg.norm(y))
        ys.append(y)
        changes.append(ch)
        print(f"mu={mu} spin={spin} colour={colour}: k_used={kr.k_used} change from k={kc}: {ch:.2e} "
              f"({time.time() - t:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "point4_full_10x4.npz"), y=np.array(ys),
                        mu=np.array([s[0] for s in SOURCES]), spin=np.array([s[1] for s in SOURCES]),
                        colour=np.array([s[2] for s in SOURCES]), change_from_k_check=np.array(changes),
                        k_ref=np.array([K_REF[s[0]] for s in SOURCES]))


if __name__ == "__main__":
    main()
