"""GPU tests of the learned ell/k policy machinery: the label runs against the
oracle's nested coefficients, and the predict / verify / fall-back logic
driven by hand-set constant networks (so the outcome does not depend on
training)."""
import functools
import math

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, lattice, operator, rel, to_np

pytestmark = pytest.mark.gpu

DOUBLING, LEARNED = 1, 2
DIMS, EPS, SEED, SRC = (4, 4, 4, 4), 0.5, 4401, 4402


def constant_net(k_star, ell_star):
    """A network whose output is (log10 k_star, log10 ell_star) for any input."""
    from paper_0912_4457_amd import policy as P
    params = np.zeros(P.NPARAMS, np.float32)
    params[-2:] = [math.log10(k_star), math.log10(ell_star)]
    return P.pack(params, np.zeros(16), np.ones(16), np.zeros(2), np.ones(2))


@functools.lru_cache(maxsize=None)
def exact(mu):
    from oracle import nested
    return nested.sign_exact_dense(operator(DIMS, EPS, SEED, mu), I.gaussian_source(DIMS, SRC))


@functools.lru_cache(maxsize=None)
def plain_k(mu, tol):
    import paper_0912_4457_amd as nks
    x, st = nks.sign_apply(lattice(DIMS, EPS, SEED, mu), I.gaussian_source(DIMS, SRC).ravel(), k=1000, ell=400,
                           tol=tol, k_policy=DOUBLING, ell_policy=DOUBLING)
    assert st["status"] == 0
    return st["k_used"]


def _learned(mu, tol, net):
    import paper_0912_4457_amd as nks
    c = ctx()
    nks.policy_load(c, net)
    return nks.sign_apply(lattice(DIMS, EPS, SEED, mu), I.gaussian_source(DIMS, SRC).ravel(), k=1000, ell=400,
                          tol=tol, k_policy=LEARNED, ell_policy=LEARNED)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_predicted_k_is_verified_and_accepted(mu):
    tol = 1e-9
    kp = plain_k(mu, tol)
    # a prediction at the size the plain checkpoints accepted passes verification
    x, st = _learned(mu, tol, constant_net(kp - 10, 64))
    assert st["status"] == 0, st
    assert st["k_used"] == kp
    assert st["outer_delta"] <= tol / 4
    # the inner doubling started at 64: 64 -> 128 (or non-nested once 2 ell covers H_k)
    assert st["ell_used"] == 0 or st["ell_used"] >= 128
    assert st["inner_delta"] <= tol / 10
    assert rel(to_np(x), exact(mu)) <= 10 * tol


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_short_prediction_falls_back_to_checkpoints(mu):
    # two-sided on this 3072-dimensional operator the weighted coefficient
    # change between checkpoints levels off near 2e-11 (k = 1000, the cap):
    # tol = 1e-10 would put the tol/4 acceptance on that rounding floor
    tol = 1e-10 if mu == 0.0 else 1e-9
    kp = plain_k(mu, tol)
    assert kp >= 300
    x, st = _learned(mu, tol, constant_net(125, 16))     # k target 140: far too short
    assert st["status"] == 0, st
    assert st["k_used"] % 100 == 0 and st["k_used"] >= 200
    assert abs(st["k_used"] - kp) <= 100
    assert rel(to_np(x), exact(mu)) <= 10 * tol


def test_prediction_beyond_k_cap_behaves_as_doubling():
    import paper_0912_4457_amd as nks
    tol = 1e-9
    kp = plain_k(0.0, tol)
    x, st = _learned(0.0, tol, constant_net(5000, 64))
    assert st["status"] == 0 and st["k_used"] == kp
    assert rel(to_np(x), exact(0.0)) <= 10 * tol
    nks.policy_load(ctx(), constant_net(300, 64))


def test_two_sided_label_runs_are_refused():
    import paper_0912_4457_amd as nks
    with pytest.raises(nks.NKSError):
        nks.policy_label([dict(lat=lattice(DIMS, EPS, SEED, 0.3), b=I.gaussian_source(DIMS, SRC).ravel(), k=200,
                               ell=64, tol=1e-8)])


def test_learned_policy_needs_a_network():
    import paper_0912_4457_amd as nks
    c = nks.Context(0)
    with pytest.raises(nks.NKSError):
        nks.sign_apply(nks.Lattice(c, DIMS, I.su3_links(DIMS, EPS, SEED)), I.gaussian_source(DIMS, SRC).ravel(),
                       k=400, ell=64, tol=1e-8, k_policy=LEARNED, ell_policy=LEARNED)
    bad = constant_net(300, 64)
    bad[-1] = 0.0                      # a target scale of zero
    with pytest.raises(nks.NKSError):
        nks.policy_load(c, bad)


@functools.lru_cache(maxsize=None)
def _labels(mu):
    import paper_0912_4457_amd as nks
    lab = nks.policy_label([dict(lat=lattice(DIMS, EPS, SEED, mu), b=I.gaussian_source(DIMS, SRC).ravel(), k=400,
                                 ell=512, tol=1e-8)])
    return lab[0]


@functools.lru_cache(maxsize=None)
def _ritz(mu, k):
    from oracle import krylov
    op = operator(DIMS, EPS, SEED, mu)
    b = I.gaussian_source(DIMS, SRC).ravel()
    if mu == 0.0:
        return krylov.lanczos(op.matvec, b, k)
    return krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, k)


TWO_SIDED_LABEL_OFF = pytest.mark.skip(
    reason="two-sided label runs faulted the GPU (memory aperture violation in the label kernel, "
           "4^4 mu=0.3 k=400); switched off in nks_policy_label until the cause is shown")


@pytest.mark.parametrize("mu", [0.0, pytest.param(0.3, marks=TWO_SIDED_LABEL_OFF)])
def test_label_errors_match_oracle(mu):
    from oracle import policy
    from paper_0912_4457_amd import policy as P
    row = _labels(mu)
    kr = _ritz(mu, 400)
    herm = mu == 0.0
    vnorm = np.linalg.norm(kr.V, axis=0)
    c_ref, _ = policy.ell_doubling(kr.alpha, kr.beta, kr.gamma, herm, 1e-13, ell_max=512)
    e = row[P.NFEAT:P.NFEAT + P.LABEL_NK]
    ks = P.LABEL_DK * (np.arange(P.LABEL_NK) + 1)
    assert np.all(np.isfinite(e[ks <= 400])) and np.all(np.isnan(e[ks > 400]))
    assert e[ks == 400][0] == 0.0
    # The two-sided recurrence loses biorthogonality: beyond about 200 steps at
    # this roughness its H_k depends on rounding (a 1e-15 change of b moves
    # e(240) by 10% in the oracle itself), so the GPU's and the oracle's H_k
    # are compared only where they still agree.
    for k in ((100, 160, 240, 320) if herm else (60, 100, 160, 200)):
        c, _ = policy.ell_doubling(kr.alpha[:k], kr.beta[:k - 1], kr.gamma[:k - 1], herm, 1e-13, ell_max=512)
        d = c_ref.copy()
        d[:k] -= c
        e_ref = policy.weighted_norm(d, vnorm) / policy.weighted_norm(c_ref, vnorm)
        got = e[k // P.LABEL_DK - 1]
        assert got == pytest.approx(e_ref, rel=0.05 if herm else 0.01, abs=1e-11), k
    # doubling trace: finite changes that shrink until the doubling stops
    tr = row[P.NFEAT + P.LABEL_NK:].reshape(P.LABEL_NK, P.LABEL_NELL)
    t = tr[ks == 320][0]
    fin = t[np.isfinite(t)]
    assert fin.size >= 1 and np.all(fin >= 0)


@pytest.mark.parametrize("mu", [0.0, pytest.param(0.3, marks=TWO_SIDED_LABEL_OFF)])
def test_label_features_match_oracle(mu):
    from paper_0912_4457_amd import policy as P
    f = _labels(mu)[:P.NFEAT]
    kr = _ritz(mu, 100)
    herm = mu == 0.0
    from oracle import nested
    H = kr.H()
    zmin, zmax = nested.ritz_extremes(np.diag(H), np.diag(H, -1), np.diag(H, 1), herm)
    zmin2, _ = nested.ritz_extremes(np.diag(H)[:50], np.diag(H, -1)[:49], np.diag(H, 1)[:49], herm)
    tol_log = 0.0 if herm else 0.1     # two-sided extremes are power-iteration estimates
    assert f[0] == 1.0
    assert f[1] == pytest.approx(math.log10(zmin), abs=tol_log + 1e-6)
    assert f[2] == pytest.approx(math.log10(zmax), abs=tol_log + 1e-6)
    assert f[3] == pytest.approx(math.log10(zmin2), abs=tol_log + 1e-6)
    assert f[4] == pytest.approx(f[2] - f[1], abs=1e-12)
    assert f[5] == pytest.approx(mu) and f[6] == pytest.approx(-8.0)
    assert f[7] == (0.0 if herm else 1.0) and f[8] == pytest.approx(math.log10(256))
    assert f[9] == pytest.approx(np.mean(np.abs(kr.alpha)), rel=1e-9)
    assert f[10] == pytest.approx(np.mean(np.sqrt(np.abs(kr.beta * kr.gamma))), rel=1e-9)
    assert np.all(f[11:] == 0.0)


# ---------------------------------------------------------------- trained network
def _held_out_configs():
    """Lattices the shipped network never saw (its training used seed 31 and
    sample_configs draws seeds seed * 1000 + i), small enough for the oracle."""
    from paper_0912_4457_amd import policy as P
    cfgs = [c for c in P.sample_configs(40, 33) if np.prod(c["dims"]) <= 4096 and c["eps"] <= 0.38]
    return cfgs[:4]


@functools.lru_cache(maxsize=None)
def _oracle_reference(i):
    from oracle import dirac, policy
    c = _held_out_configs()[i]
    op = dirac.Operator(I.su3_links(c["dims"], c["eps"], c["seed"]), c["dims"], c["m0"], c["mu"])
    b = _source(c)
    y, info = policy.sign_apply_policy(op, b, 1e-12, k_max=1600, ell_max=256)
    return y.ravel(), info


def _source(c):
    rng = np.random.default_rng(c["seed"] + 5)
    return I.point_source(c["dims"], int(rng.integers(4)), int(rng.integers(3)),
                          int(rng.integers(int(np.prod(c["dims"])))))


def test_trained_network_gains_over_doubling():
    """The shipped network against the plain policies on held-out lattices:
    same accuracy against the oracle, less device time."""
    import paper_0912_4457_amd as nks
    c0 = ctx()
    meta = nks.load_policy(c0)
    assert meta["samples_train"] > 1000
    rows = []
    for i, c in enumerate(_held_out_configs()):
        lat = nks.Lattice(c0, c["dims"], I.su3_links(c["dims"], c["eps"], c["seed"]), m0=c["m0"], mu=c["mu"])
        b = _source(c).ravel()
        y_ref, info = _oracle_reference(i)
        assert info["converged"]
        for tol in (1e-8, 1e-10):
            r = {}
            for name, pol in (("plain", DOUBLING), ("learned", LEARNED)):
                nks.sign_apply(lat, b, k=1400, ell=256, tol=tol, k_policy=pol, ell_policy=pol)   # warm-up
                x, st = nks.sign_apply(lat, b, k=1400, ell=256, tol=tol, k_policy=pol, ell_policy=pol)
                assert st["status"] == 0, (c, tol, name, st)
                err = rel(to_np(x), y_ref)
                assert err <= 10 * tol, (c, tol, name, err)
                r[name] = (st["k_used"], st["ms_outer"] + st["ms_nested"] + st["ms_lift"], err)
            rows.append((c["dims"], c["mu"], tol, r))
        lat.close()
    ms_plain = sum(r["plain"][1] for *_, r in rows)
    ms_learned = sum(r["learned"][1] for *_, r in rows)
    for dims, mu, tol, r in rows:
        print(f"{dims} mu={mu} tol={tol:g}: k {r['plain'][0]} -> {r['learned'][0]}, "
              f"ms {r['plain'][1]:.1f} -> {r['learned'][1]:.1f}, err {r['plain'][2]:.1e} / {r['learned'][2]:.1e}")
    print(f"device time plain {ms_plain:.1f} ms, learned {ms_learned:.1f} ms ({ms_learned / ms_plain:.2f})")
    assert ms_learned <= 0.85 * ms_plain
