"""Write tests/golden/point12_10x4_sketch.npz: a full-vector check of the
benchmark's 24 results (10^4 lattice, eps = 0.35, link seed 10401, m0 = 1.6,
the 12 spin-colour point sources at mu = 0 and mu = 0.2) that needs 256
numbers per source instead of 120000.

For each source the oracle's converged reference y (the non-nested
Krylov-Ritz result with the spectral sign of H_k at k = 1400 / 1000, as in
make_point12_10x4.py) is stored as S y, with S the 256-row seeded complex
Gaussian sketch of ``nks_inputs.sketch_rows``, together with |y|: then
|S x - S y| / (16 |y|) estimates the full-vector relative error of any
result x to about 3 %.  The file also holds the oracle's own full-vector
errors (exact, not sketched) at outer sizes k = 440 ... 700, without nesting
and with the nested method at ell = 64 (p as in a sign application), which fix the smallest k at which the
method itself reaches a given accuracy on this workload.

Calls only ``oracle`` and ``nks_inputs``.  About an hour with 5 single-threaded
workers.  Usage: python tests/golden/make_sketch_10x4.py [--workers N]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import nks_inputs as I  # noqa: E402
from make_point12_10x4 import DIMS, K_CHECK, K_REF, sign_e1  # noqa: E402
from oracle import dirac, krylov, nested  # noqa: E402

ROWS, SEED = 256, 20261204
KS = tuple(range(440, 701, 20))
ELL = 64


def one_source(case):
    """Reference, its sketch and the oracle's errors at KS for one source."""
    mu, spin, colour = case
    t = time.time()
    n = 12 * I.volume(DIMS)
    op = dirac.Operator(I.su3_links(DIMS, 0.35, 10401), DIMS, 1.6, mu)
    herm = mu == 0.0
    b = I.point_source(DIMS, spin, colour).ravel()
    if herm:
        kr = krylov.lanczos(op.matvec, b, K_REF[mu])
    else:
        kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, K_REF[mu])
    y = kr.bnorm * (kr.V @ sign_e1(kr.alpha, kr.beta, kr.gamma, herm))
    ny = float(np.linalg.norm(y))
    kc = min(K_CHECK[mu], kr.k_used)
    y2 = kr.bnorm * (kr.V[:, :kc] @ sign_e1(kr.alpha[:kc], kr.beta[:kc - 1], kr.gamma[:kc - 1], herm))
    change = float(np.linalg.norm(y - y2)) / ny
    e_plain, e_nested = [], []
    for k in KS:
        a, be, ga = kr.alpha[:k], kr.beta[:k - 1], kr.gamma[:k - 1]
        yk = kr.bnorm * (kr.V[:, :k] @ sign_e1(a, be, ga, herm))
        e_plain.append(float(np.linalg.norm(yk - y)) / ny)
        c, _ = nested.nested_coefficients(a, be, ga, herm, ELL, zmax_bound=op.norm_bound)
        e_nested.append(float(np.linalg.norm(kr.bnorm * (kr.V[:, :k] @ c) - y)) / ny)
    sy = I.sketch_rows(n, range(ROWS), SEED) @ y
    print(f"mu={mu} spin={spin} colour={colour}: change {change:.1e}, nested ell={ELL} errors "
          + " ".join(f"{k}:{e:.1e}" for k, e in zip(KS, e_nested)) + f" ({time.time() - t:.0f} s)", flush=True)
    return sy, ny, change, e_plain, e_nested


def _single_thread():
    for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"


def main():
    import multiprocessing as mp
    workers = int(sys.argv[sys.argv.index("--workers") + 1]) if "--workers" in sys.argv else 4
    cases = [(mu, spin, colour) for mu in (0.0, 0.2) for spin in range(4) for colour in range(3)]
    # the slow two-sided sources first, so the pool's tail is short
    order = sorted(range(len(cases)), key=lambda i: -cases[i][0])
    _single_thread()                                  # inherited by the spawned workers
    with mp.get_context("spawn").Pool(workers) as pool:
        res = dict(zip(order, pool.map(one_source, [cases[i] for i in order], chunksize=1)))
    out = [res[i] for i in range(len(cases))]
    np.savez_compressed(os.path.join(HERE, "point12_10x4_sketch.npz"), rows=ROWS, seed=SEED,
                        mu=np.array([c[0] for c in cases]), spin=np.array([c[1] for c in cases]),
                        colour=np.array([c[2] for c in cases]), sy=np.array([o[0] for o in out]),
                        norm=np.array([o[1] for o in out]), change_from_k_check=np.array([o[2] for o in out]),
                        ks=np.array(KS), ell=ELL, oracle_err_plain=np.array([o[3] for o in out]),
                        oracle_err_nested=np.array([o[4] for o in out]))


if __name__ == "__main__":
    main()
