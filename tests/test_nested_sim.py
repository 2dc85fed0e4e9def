"""The nested-step kernels' device code (nested.hip) run on the CPU under an
emulation of the HIP thread model (tests/cpu_sim) with AddressSanitizer:
its results against the oracle's nested step (App. C steps 3-5, Eq. nested),
and every memory access it makes checked, without a GPU."""
import functools
import os
import shutil
import sys

import numpy as np
import pytest

import nks_inputs as I
from oracle import dirac, krylov, nested, policy

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpu_sim"))
import nestsim  # noqa: E402

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")

DIMS, EPS, SEED, SRC = (4, 4, 4, 4), 0.5, 4401, 4402


@functools.lru_cache(maxsize=None)
def _exe(tmp_root):
    os.makedirs(tmp_root, exist_ok=True)
    return nestsim.build(tmp_root, asan=True)


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return _exe(str(tmp_path_factory.mktemp("nestsim")))


@functools.lru_cache(maxsize=None)
def _krylov(mu, k):
    op = dirac.Operator(I.su3_links(DIMS, EPS, SEED), DIMS, 1.6, mu)
    b = I.gaussian_source(DIMS, SRC).ravel()
    if mu == 0.0:
        return krylov.lanczos(op.matvec, b, k)
    return krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, k)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_emulated_nested_step_matches_oracle(exe, mu):
    """Fixed (k, ell, p): the kernel's c = sgn(H_k') restricted to the inner
    space equals the oracle's to rounding (same steps, same LAPACK pivoting)."""
    k, ell = 40, 16
    kr = _krylov(mu, k)
    herm = mu == 0.0
    c_or, info = nested.nested_coefficients(kr.alpha, kr.beta, kr.gamma, herm, ell, p=None)
    r = nestsim.run(exe, kr.alpha, kr.beta, kr.gamma, herm, ell, p=info["p"])
    assert r["status"][nestsim.ST_STATUS] == 0 and r["status"][nestsim.ST_ELL] == ell
    err = np.linalg.norm(r["c"] - c_or) / np.linalg.norm(c_or)
    print(f"mu={mu}: emulated nested step vs oracle {err:.2e}")
    assert err < 1e-12


def test_emulated_label_run_is_in_bounds_and_matches_oracle(exe):
    """A two-sided label run (features, reference c, three label points with
    ell doubling up to the non-nested RHi) under AddressSanitizer, each label
    point's nested scratch area the only one left unpoisoned; its label
    errors against the oracle's doubling at the same k.  Label runs need at
    least 120 outer vectors (the features take H_100)."""
    k = 120
    kr = _krylov(0.3, k)
    vn = np.linalg.norm(kr.V, axis=0)
    c_ref, _ = policy.ell_doubling(kr.alpha, kr.beta, kr.gamma, False, 1e-13, ell_max=2 * k)
    r = nestsim.run(exe, kr.alpha, kr.beta, kr.gamma, False, 2 * k, vnorm=vn, mode=nestsim.NEST_LABEL,
                    label_points=(0, 3), tol=1e-8)
    assert "AddressSanitizer" not in r["log"]
    lab = r["label"]
    for i in range(3):
        ki = nestsim.LABEL_DK * (i + 1)
        c, _ = policy.ell_doubling(kr.alpha[:ki], kr.beta[:ki - 1], kr.gamma[:ki - 1], False, 1e-13,
                                   ell_max=2 * k)
        d = c_ref.copy()
        d[:ki] -= c
        e_ref = policy.weighted_norm(d, vn) / policy.weighted_norm(c_ref, vn)
        got = lab[nestsim.NFEAT + i]
        print(f"k_i={ki}: label error {got:.3e} oracle {e_ref:.3e}")
        assert got == pytest.approx(e_ref, rel=1e-6, abs=1e-13)
    assert np.all(np.isnan(lab[nestsim.NFEAT + 3:nestsim.NFEAT + nestsim.LABEL_NK]))   # points not run
