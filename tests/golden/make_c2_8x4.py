"""Write tests/golden/c2_8x4.npz: references for sgn(A) b on the 8^4 lattice
of the two-sided workload (SU(3) links eps = 0.4, seed 8401, m0 = 1.6,
mu = 0.3, Gaussian source seed 8402).  At k = 800 this workload is far from
converged without deflation (near-critical links), so:

* the M eigenpairs of A of smallest |lambda|, right ones from A and left ones
  from A^dagger, by ARPACK in shift-invert mode around 0 on the oracle's CSR
  (one sparse LU of A serves both), paired by eigenvalue and scaled to
  l_i^dagger r_i = 1, with the pins that certify them: the residuals of both eigen-equations (unit
  vectors) and the biorthonormality |l_i^dagger r_j - delta_ij|;
* y_ref, the converged result: sum_i sgn(Re lambda_i) <l_i, b> r_i plus the
  non-nested Krylov-Ritz result on the deflated source (App. C steps 1 and
  6, Eq. non-nested-oblique, spectral sign of H_k) at k = K_REF, with its
  change from k = K_CHECK as its accuracy;
* the oracle's nested method at the workload's k = 800, ell = 150: with the
  same deflation (its distance to y_ref is the method's own error there), and
  without (y_run, the element-wise target of the GPU's run at the same k,
  ell, p, with the oracle's response to two-ulp changes of the source as the
  scale of rounding differences).

Calls only ``oracle``, ``nks_inputs`` and scipy.  About half an hour.
Usage: python tests/golden/make_c2_8x4.py
"""
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)
os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")

import nks_inputs as I  # noqa: E402
from make_point12_10x4 import sign_e1  # noqa: E402
from oracle import deflation, dirac, krylov, nested  # noqa: E402

DIMS, EPS, SEED, M0, MU, SRC = (8, 8, 8, 8), 0.4, 8401, 1.6, 0.3, 8402
M = 16
K_REF, K_CHECK = 1400, 1100
K_RUN, ELL_RUN = 800, 150


def smallest_eigs(solve, n, m):
    """m eigenpairs of the matrix whose inverse ``solve`` applies, with the
    smallest |lambda| (ARPACK on the inverse, i.e. shift-invert at 0)."""
    inv = spla.LinearOperator((n, n), matvec=solve, dtype=np.complex128)
    w, v = spla.eigs(inv, k=m, which="LM", ncv=4 * m, tol=1e-12, maxiter=5000)
    lam = 1.0 / w
    idx = np.argsort(np.abs(lam))
    v = v[:, idx]
    return lam[idx], (v / np.linalg.norm(v, axis=0)).T.copy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def main():
    t0 = time.time()
    op = dirac.Operator(I.su3_links(DIMS, EPS, SEED), DIMS, M0, MU)
    b = I.gaussian_source(DIMS, SRC).ravel()
    n = op.A.shape[0]
    lu = spla.splu(op.A.tocsc(), permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))
    print(f"sparse LU {time.time() - t0:.0f} s", flush=True)
    lam_r, r = smallest_eigs(lu.solve, n, M)
    # left eigenvectors: right ones of A^dagger (eigenvalues conj(lambda)), same factors
    lam_l, l = smallest_eigs(lambda x: lu.solve(x, trans="H"), n, M)
    del lu
    print(f"eigs {time.time() - t0:.0f} s, |lambda| {abs(lam_r[0]):.3e} .. {abs(lam_r[-1]):.3e}", flush=True)
    # pair left with right by eigenvalue, scale to l^dagger r = 1
    order = [int(np.argmin(np.abs(np.conj(lam_l) - lr))) for lr in lam_r]
    assert len(set(order)) == M, "left and right eigenvalues do not pair up"
    l = l[order]
    pair_gap = float(np.max(np.abs(np.conj(lam_l[order]) - lam_r)))
    for i in range(M):
        l[i] = l[i] / np.conj(np.vdot(l[i], r[i]))
    res_r = max(float(np.linalg.norm(op.matvec(r[i]) - lam_r[i] * r[i])) for i in range(M))
    res_l = max(float(np.linalg.norm(op.rmatvec(l[i]) - np.conj(lam_r[i]) * l[i]) / np.linalg.norm(l[i]))
                for i in range(M))
    biorth = float(np.max(np.abs(np.conj(l) @ r.T - np.eye(M))))
    print(f"residuals right {res_r:.1e} left {res_l:.1e}, biorthonormality {biorth:.1e}, pairing {pair_gap:.1e}",
          flush=True)
    xm, d = deflation.project(b, r, l)
    low = (np.sign(np.real(lam_r)) * d) @ r
    kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, xm, K_REF)
    y = kr.bnorm * (kr.V @ sign_e1(kr.alpha, kr.beta, kr.gamma, False)) + low
    kc = min(K_CHECK, kr.k_used)
    y2 = kr.bnorm * (kr.V[:, :kc] @ sign_e1(kr.alpha[:kc], kr.beta[:kc - 1], kr.gamma[:kc - 1], False)) + low
    change = rel(y2, y)
    del kr
    print(f"reference k_ref={K_REF}, change from k={kc}: {change:.2e} ({time.time() - t0:.0f} s)", flush=True)
    y_defl, _ = deflation.sign_apply_deflated(op, b, K_RUN, ELL_RUN, r, l, lam_r)
    e_defl = rel(y_defl, y)
    y_run, info = nested.sign_apply(op, b, K_RUN, ELL_RUN)
    e_run = rel(y_run, y)
    resp = 0.0
    for s in range(3):
        rng = np.random.default_rng(7100 + s)
        rms = float(np.linalg.norm(b)) / np.sqrt(b.size)
        bp = b * (1 + 4e-16 * rng.choice([-1.0, 1.0], b.shape)) + 4e-16 * rms * rng.choice([-1.0, 1.0], b.shape)
        resp = max(resp, rel(nested.sign_apply(op, bp, K_RUN, ELL_RUN, p=info["p"])[0], y_run))
    print(f"oracle at k={K_RUN} ell={ELL_RUN}: deflated {e_defl:.2e}, plain {e_run:.2e} from the reference; "
          f"plain run's rounding response {resp:.2e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_8x4.npz"), y_ref=y, lam=lam_r, change_from_k_check=change,
                        k_ref=K_REF, k_check=kc, resid_right=res_r, resid_left=res_l, biorth=biorth,
                        oracle_err_deflated=e_defl, y_run=np.ravel(y_run), p_run=info["p"],
                        oracle_err_run=e_run, run_rounding_response=resp, k_run=K_RUN, ell_run=ELL_RUN, m=M)


if __name__ == "__main__":
    main()
