"""Write tests/golden/uneven64_sketch.npz: converged references for the 64 jobs
of the benchmark's uneven batch (point sources drawn with seed 64 over nine
lattices: 6^4, 8^4 and 10^4, eps = 0.35, link seeds 6601 / 8801 / 10401,
m0 = 1.6, each at mu in {0, 0.1, 0.3}; tolerance 1e-6 or 1e-8 per job), stored
as 256-row Gaussian sketches (``nks_inputs.sketch_rows``, one sketch matrix
per lattice size) with the reference norms, so that the full-vector error of
every batched result can be estimated to about 3 %.

Reference: the non-nested Krylov-Ritz result with the spectral sign of H_k
(Eqs. non-nested / non-nested-oblique) at k = 1400 (Lanczos) or 1000
(two-sided), its change from k = 1100 / 800 stored as its accuracy.  The job list repeats the benchmark's draws
in the same order.

Calls only ``oracle`` and ``nks_inputs``.  About an hour with 4 single-threaded
workers.  Usage: python tests/golden/make_uneven_sketch.py [--workers N]
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
from make_point12_10x4 import sign_e1  # noqa: E402
from oracle import dirac, krylov  # noqa: E402

EPS, M0 = 0.35, 1.6
LATS = (((6, 6, 6, 6), 6601), ((8, 8, 8, 8), 8801), ((10, 10, 10, 10), 10401))
MUS = (0.0, 0.1, 0.3)
ROWS, SEED = 256, 20261205
K_REF = {True: 1400, False: 1000}      # Lanczos / two-sided (which drifts beyond 1000)
K_CHECK = {True: 1100, False: 800}


def jobs():
    """(lattice index, dims, link seed, mu, spin, colour, site, tol) for the 64
    jobs, drawn as the benchmark draws them."""
    rng = np.random.default_rng(64)
    lats = [(dims, seed, mu) for dims, seed in LATS for mu in MUS]
    out = []
    for i in range(64):
        li = i % len(lats)
        dims, seed, mu = lats[li]
        spin, colour = int(rng.integers(4)), int(rng.integers(3))
        site = int(rng.integers(I.volume(dims)))
        tol = float(rng.choice([1e-6, 1e-8]))
        out.append((li, dims, seed, mu, spin, colour, site, tol))
    return out


def one_job(job):
    """Sketch, norm and accuracy of one job's converged reference."""
    li, dims, seed, mu, spin, colour, site, tol = job
    t = time.time()
    n = 12 * I.volume(dims)
    op = dirac.Operator(I.su3_links(dims, EPS, seed), dims, M0, mu)
    herm = mu == 0.0
    b = I.point_source(dims, spin, colour, site).ravel()
    kr = krylov.lanczos(op.matvec, b, K_REF[herm]) if herm else \
        krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, K_REF[herm])
    y = kr.bnorm * (kr.V @ sign_e1(kr.alpha, kr.beta, kr.gamma, herm))
    kc = min(K_CHECK[herm], kr.k_used)
    y2 = kr.bnorm * (kr.V[:, :kc] @ sign_e1(kr.alpha[:kc], kr.beta[:kc - 1], kr.gamma[:kc - 1], herm))
    ny = float(np.linalg.norm(y))
    change = float(np.linalg.norm(y - y2)) / ny
    sy = I.sketch_rows(n, range(ROWS), SEED) @ y
    print(f"{dims} mu={mu} source ({spin},{colour}) at {site}, tol {tol:g}: change {change:.1e} "
          f"({time.time() - t:.0f} s)", flush=True)
    return sy, ny, change


def main():
    import multiprocessing as mp
    workers = int(sys.argv[sys.argv.index("--workers") + 1]) if "--workers" in sys.argv else 4
    js = jobs()
    for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"                          # inherited by the spawned workers
    # largest lattices and two-sided jobs first, so the pool's tail is short
    order = sorted(range(len(js)), key=lambda i: (-I.volume(js[i][1]), -js[i][3]))
    with mp.get_context("spawn").Pool(workers) as pool:
        res = dict(zip(order, pool.map(one_job, [js[i] for i in order], chunksize=1)))
    out = [res[i] for i in range(len(js))]
    np.savez_compressed(os.path.join(HERE, "uneven64_sketch.npz"), rows=ROWS, seed=SEED,
                        lattice=np.array([j[0] for j in js]), mu=np.array([j[3] for j in js]),
                        spin=np.array([j[4] for j in js]), colour=np.array([j[5] for j in js]),
                        site=np.array([j[6] for j in js]), tol=np.array([j[7] for j in js]),
                        sy=np.array([o[0] for o in out]), norm=np.array([o[1] for o in out]),
                        change_from_k_check=np.array([o[2] for o in out]),
                        k_ref=np.array([K_REF[j[3] == 0.0] for j in js]),
                        k_check=np.array([K_CHECK[j[3] == 0.0] for j in js]))


if __name__ == "__main__":
    main()
