"""GPU parity of the deflated sign application (App. C steps 1 and 6) with
eigenpairs from a dense eigendecomposition: against the oracle at the same
(k, ell, p), the gain in accuracy over the undeflated method, and the error
paths."""
import functools

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import lattice, operator, rel, rounding_tolerance, to_np

pytestmark = pytest.mark.gpu

CASES = {0.0: ((4, 4, 4, 4), 16), 0.3: ((3, 3, 3, 3), 12)}


@functools.lru_cache(maxsize=None)
def _pairs(mu):
    from oracle import deflation
    dims, m = CASES[mu]
    return deflation.eigenpairs_smallest(operator(dims, 0.5, 4401, mu), m)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_deflated_sign_matches_oracle_same_parameters(mu):
    import paper_0912_4457_amd as nks
    from oracle import deflation, nested
    dims, m = CASES[mu]
    lam, r, l = _pairs(mu)
    op = operator(dims, 0.5, 4401, mu)
    lat = lattice(dims, 0.5, 4401, mu)
    b = I.gaussian_source(dims, 4402).ravel()
    xm, _ = deflation.project(b, r, l)
    _, info = nested.sign_apply(op, xm, 100, 30)
    ref, _ = deflation.sign_apply_deflated(op, b, 100, 30, r, l, lam, p=info["p"])
    lat.set_deflation(r, lam, None if mu == 0.0 else l)
    try:
        x, st = nks.sign_apply(lat, b, k=100, ell=30, p=info["p"], deflate=True)
    finally:
        lat.set_deflation(None, [])
    assert st["status"] == 0
    err = rel(to_np(x), ref)
    tol, resp = rounding_tolerance(
        lambda v: deflation.sign_apply_deflated(op, v, 100, 30, r, l, lam, p=info["p"])[0], b, mu == 0.0)
    print(f"mu={mu}: deflated sign vs oracle (same k, ell, p, eigenpairs) {err:.2e}, tolerance {tol:.1e} "
          f"(oracle's rounding response {resp:.1e})")
    assert err <= tol


def test_deflation_improves_accuracy_at_fixed_k():
    import paper_0912_4457_amd as nks
    from oracle import nested
    dims, m = CASES[0.0]
    lam, r, l = _pairs(0.0)
    lat = lattice(dims, 0.5, 4401, 0.0)
    b = I.gaussian_source(dims, 4402).ravel()
    exact = nested.sign_exact_dense(operator(dims, 0.5, 4401, 0.0), b)
    x0, _ = nks.sign_apply(lat, b, k=120, ell=120)
    lat.set_deflation(r, lam)
    try:
        x1, st = nks.sign_apply(lat, b, k=120, ell=120, deflate=True)
    finally:
        lat.set_deflation(None, [])
    assert st["status"] == 0
    e0, e1 = rel(to_np(x0), exact), rel(to_np(x1), exact)
    print(f"k=120: error without deflation {e0:.2e}, with 16 deflated eigenpairs {e1:.2e}")
    assert e1 < 0.2 * e0


def test_deflation_errors():
    import paper_0912_4457_amd as nks
    dims, _ = CASES[0.0]
    lat = lattice(dims, 0.5, 4401, 0.0)
    b = I.gaussian_source(dims, 4402).ravel()
    with pytest.raises(nks.NKSError):                      # no eigenpairs set
        nks.sign_apply(lat, b, k=40, ell=10, deflate=True)
    r = np.zeros((1, lat.n), np.complex128)
    r[0, 0] = 1.0
    with pytest.raises(nks.NKSError):                      # sgn undefined for Re(lambda) = 0
        lat.set_deflation(r, [0.5j])
    with pytest.raises(nks.NKSError):                      # too many
        lat.ctx.check(nks.lib().nks_lattice_set_deflation(lat.h, 65, None, None, None))
