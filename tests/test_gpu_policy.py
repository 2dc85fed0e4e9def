"""GPU parity of the plain tolerance-driven policies: ell-doubling in the
nested step and k-checkpoints in the outer loop, against the oracle's
policy (the same rules written independently)."""
import functools

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import M0, ctx, lattice, operator, rel, to_np

pytestmark = pytest.mark.gpu

DOUBLING = 1


@functools.lru_cache(maxsize=None)
def ritz(mu):
    from oracle import krylov
    op = operator((4, 4, 4, 4), 0.5, 4401, mu)
    b = I.gaussian_source((4, 4, 4, 4), 4402).ravel()
    if mu == 0.0:
        return krylov.lanczos(op.matvec, b, 400)
    return krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, 400)


@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_ell_doubling_matches_oracle(mu, tol):
    import paper_0912_4457_amd as nks
    from oracle import nested, policy
    kr = ritz(mu)
    herm = mu == 0.0
    _, info0 = nested.nested_coefficients(kr.alpha, kr.beta, kr.gamma, herm, 16)
    p = info0["p"]
    c_ref, info = policy.ell_doubling(kr.alpha, kr.beta, kr.gamma, herm, tol, p=p)
    c_gpu, st = nks.nested_step(ctx(), kr.alpha, kr.beta, kr.gamma, herm, 400, p=p,
                                ell_policy=DOUBLING, tol=tol)
    assert st["ell_used"] == (info["ell"] if info["nested"] else 0)
    # inner_delta = |c_2ell - c_ell| / |c_2ell| is a difference of two coefficient
    # vectors, each held to ctol of the oracle's below: it can differ by 2 ctol
    ctol = 1e-11 if herm else 1e-9
    assert st["inner_delta"] == pytest.approx(info["inner_delta"], rel=1e-3, abs=2 * ctol)
    assert rel(c_gpu, c_ref) <= ctol


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_k_checkpoints_reach_tolerance_4x4(mu):
    import paper_0912_4457_amd as nks
    from oracle import nested
    dims = (4, 4, 4, 4)
    lat = lattice(dims, 0.5, 4401, mu)
    op = operator(dims, 0.5, 4401, mu)
    b = I.gaussian_source(dims, 4402)
    ref = nested.sign_exact_dense(op, b)
    ks = []
    for tol in (1e-5, 1e-9):
        x, st = nks.sign_apply(lat, b.ravel(), k=1000, ell=400, tol=tol, k_policy=DOUBLING,
                               ell_policy=DOUBLING)
        assert st["status"] == 0, st
        assert st["k_used"] % 100 == 0 and st["outer_delta"] <= tol / 4
        assert rel(to_np(x), ref) <= 10 * tol
        ks.append(st["k_used"])
    assert ks[0] < ks[1]


def test_k_checkpoints_same_k_as_oracle():
    import paper_0912_4457_amd as nks
    from oracle import policy
    dims = (4, 4, 4, 4)
    lat = lattice(dims, 0.5, 4401, 0.0)
    op = operator(dims, 0.5, 4401, 0.0)
    b = I.gaussian_source(dims, 4402)
    tol = 1e-7
    y_ref, info = policy.sign_apply_policy(op, b, tol, k_max=1000, ell_max=400)
    x, st = nks.sign_apply(lat, b.ravel(), k=1000, ell=400, tol=tol, k_policy=DOUBLING, ell_policy=DOUBLING)
    # p comes from Sturm multisection on the GPU (exact to ~1e-7), so the two
    # nested results agree to the inner tolerance, not to rounding
    assert st["k_used"] == info["k"]
    assert rel(to_np(x), y_ref) <= tol


def test_policy_at_full_size_pure_gauge():
    import paper_0912_4457_amd as nks
    from oracle import closedform
    dims = (10, 10, 10, 10)
    g = I.random_su3_field(dims, 1234)
    lat = lattice(dims, 0.0, 1234, 0.2, kind="pure")
    b = I.gaussian_source(dims, 99)
    ref = closedform.pure_gauge_sign_apply(b, g, dims, M0, 0.2)
    x, st = nks.sign_apply(lat, b.ravel(), k=800, ell=256, tol=1e-9, k_policy=DOUBLING, ell_policy=DOUBLING)
    assert st["status"] == 0
    assert rel(to_np(x), ref) <= 1e-8


def test_k_policy_not_converged_reports_noconv():
    import paper_0912_4457_amd as nks
    dims = (4, 4, 4, 4)
    lat = lattice(dims, 0.5, 4401, 0.0)
    x, st = nks.sign_apply(lat, I.gaussian_source(dims, 4402).ravel(), k=200, ell=64, tol=1e-12,
                           k_policy=DOUBLING, ell_policy=DOUBLING)
    assert st["status"] == 6 and st["k_used"] == 200
