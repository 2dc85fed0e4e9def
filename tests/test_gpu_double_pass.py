"""GPU tests of the double-pass low-memory mode (Sec. 4.4): the second pass
regenerates the outer basis bit for bit, so every result equals the
single-pass one exactly (both precisions, both recurrences, with the
overlap, deflation, multi-level and k-policy options); against the oracle
at the same parameters; degenerate sources; the workspace shrinks from
O(n k) to O(n); and a 16^4 lattice against the pure-gauge closed form."""
import ctypes
import functools

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, lattice, operator, rel, rounding_tolerance, to_np

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)


def _pairs_of_runs(jobs):
    import paper_0912_4457_amd as nks
    both = []
    for j in jobs:
        both.append(dict(j, double_pass=False))
        both.append(dict(j, double_pass=True))
    xs, sts = nks.sign_apply_batch(both)
    for i in range(0, len(both), 2):
        assert sts[i]["status"] == sts[i + 1]["status"] == 0
        assert sts[i]["k_used"] == sts[i + 1]["k_used"]
        assert np.array_equal(to_np(xs[i]), to_np(xs[i + 1])), (i, rel(to_np(xs[i + 1]), to_np(xs[i])))
    return xs, sts


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_double_pass_equals_single_pass_bitwise(precision):
    la = lattice(DIMS, 0.5, 4401, 0.0)
    lb = lattice(DIMS, 0.5, 4401, 0.3)
    jobs = [dict(lat=la, b=I.gaussian_source(DIMS, 1).ravel(), k=150, ell=40),
            dict(lat=la, b=I.point_source(DIMS, 2, 1).ravel(), k=151, ell=30),      # odd k -> 152
            dict(lat=lb, b=I.gaussian_source(DIMS, 3).ravel(), k=120, ell=40),
            dict(lat=lb, b=I.gaussian_source(DIMS, 4).ravel(), k=100, ell=30, overlap=True),
            dict(lat=lb, b=I.gaussian_source(DIMS, 5).ravel(), k=100, ell=30, ell_deep=[10, 4])]
    for j in jobs:
        j["precision"] = precision
    _pairs_of_runs(jobs)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_double_pass_with_k_policy_equals_single_pass(mu):
    import paper_0912_4457_amd as nks
    lat = lattice(DIMS, 0.5, 4401, mu)
    jobs = [dict(lat=lat, b=I.gaussian_source(DIMS, 4402).ravel(), k=1000, ell=400, tol=1e-8,
                 k_policy=nks.POLICY_DOUBLING, ell_policy=nks.POLICY_DOUBLING)]
    _, sts = _pairs_of_runs(jobs)
    assert sts[0]["k_used"] < 1000


@functools.lru_cache(maxsize=None)
def _pairs(mu):
    from oracle import deflation
    return deflation.eigenpairs_smallest(operator(DIMS, 0.5, 4401, mu), 8)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_double_pass_with_deflation_equals_single_pass(mu):
    lat = lattice(DIMS, 0.5, 4401, mu)
    lam, r, l = _pairs(mu)
    lat.set_deflation(r, lam, None if mu == 0.0 else l)
    try:
        _pairs_of_runs([dict(lat=lat, b=I.gaussian_source(DIMS, 21).ravel(), k=100, ell=30, deflate=True)])
    finally:
        lat.set_deflation(None, [])


@pytest.mark.parametrize("mu,k,ell", [(0.0, 200, 50), (0.3, 200, 60)])
def test_double_pass_matches_oracle(mu, k, ell):
    import paper_0912_4457_amd as nks
    from oracle import nested
    lat = lattice(DIMS, 0.5, 4401, mu)
    op = operator(DIMS, 0.5, 4401, mu)
    b = I.gaussian_source(DIMS, 4402)
    y_ref, info = nested.sign_apply(op, b, k, ell)
    x, st = nks.sign_apply(lat, b.ravel(), k=k, ell=ell, p=info["p"], double_pass=True)
    assert st["status"] == 0 and st["k_used"] == info["k"]
    err = rel(to_np(x), y_ref)
    tol, resp = rounding_tolerance(lambda v: nested.sign_apply(op, v, k, ell, p=info["p"])[0], b, mu == 0.0)
    print(f"mu={mu} k={k} ell={ell}: double pass vs oracle (same k, ell, p) {err:.2e}, tolerance {tol:.1e} "
          f"(oracle's rounding response {resp:.1e})")
    assert err <= tol


def test_double_pass_degenerate_sources():
    import paper_0912_4457_amd as nks
    from oracle import closedform
    for mu in (0.0, 0.3):
        lat = lattice(DIMS, 0.5, 4401, mu)
        x, st = nks.sign_apply(lat, np.zeros(12 * 256, complex), k=20, ell=10, double_pass=True)
        assert st["k_used"] == 0 and np.all(to_np(x) == 0)
        x, st = nks.sign_apply(lat, np.zeros(12 * 256, complex), k=20, ell=10, double_pass=True, overlap=True)
        assert np.all(to_np(x) == 0)
    dims = (2, 2, 2, 2)
    for mu in (0.0, 0.3):                     # lucky breakdown: k_used < k
        lat = lattice(dims, 0.0, 1, mu, kind="unit")
        b = I.gaussian_source(dims, 3)
        x, st = nks.sign_apply(lat, b.ravel(), k=60, ell=60, double_pass=True)
        assert st["k_used"] < 60
        assert rel(to_np(x), closedform.free_field_sign_apply(b, dims, 1.6, mu)) <= 1e-9


def test_double_pass_workspace_is_order_n():
    # 24 jobs on 10^4 at k = 500: O(n k) basis store vs two columns per job
    import paper_0912_4457_amd as nks
    import torch
    dims = (10, 10, 10, 10)
    n = 12 * 10 ** 4
    lat = lattice(dims, 0.35, 7, 0.2)
    b = torch.zeros(n, dtype=torch.complex128, device="cuda")

    def size(double_pass):
        opts = [nks.make_opts(k=500, ell=64, double_pass=double_pass) for _ in range(24)]
        arr = (nks.Job * 24)()
        for i, o in enumerate(opts):
            arr[i].lat, arr[i].b, arr[i].x, arr[i].opts = lat.h.value, b.data_ptr(), b.data_ptr(), ctypes.pointer(o)
        sz = ctypes.c_size_t()
        ctx().check(nks.lib().nks_workspace_size(ctx().h, 24, arr, ctypes.byref(sz)))
        return sz.value

    single, double = size(False), size(True)
    assert single >= 24 * 500 * n * 16
    assert double <= 24 * 8 * n * 16
    print(f"workspace 24 jobs 10^4 k=500: single pass {single / 2**30:.1f} GiB, double pass {double / 2**30:.2f} GiB")


# the oracle's own error at these (k, ell): 5.2e-10 (mu = 0) and 1.1e-6 (mu = 0.3)
@pytest.mark.parametrize("mu,k,ell,tol", [(0.0, 200, 60, 1e-9), (0.3, 400, 100, 2e-6)])
def test_double_pass_16x4_pure_gauge_closed_form(mu, k, ell, tol):
    import paper_0912_4457_amd as nks
    from oracle import closedform
    dims = (16, 16, 16, 16)
    g = I.random_su3_field(dims, 77)
    lat = lattice(dims, 0.0, 77, mu, kind="pure")
    b = I.gaussian_source(dims, 78)
    ref = closedform.pure_gauge_sign_apply(b, g, dims, 1.6, mu)
    x, st = nks.sign_apply(lat, b.ravel(), k=k, ell=ell, double_pass=True)
    assert st["status"] == 0
    assert rel(to_np(x), ref) <= tol


def test_double_pass_and_levels_in_graph_replays_match_eager():
    # the second pass and the deeper levels inside captured graphs: every
    # replay (with eager work and synchronisation between) gives the eager bits
    import math
    import torch
    import paper_0912_4457_amd as nks
    c = nks.Context(0)
    u = I.su3_links(DIMS, 0.5, 4401)
    lats = [nks.Lattice(c, DIMS, u, mu=0.0), nks.Lattice(c, DIMS, u, mu=0.3)]
    jobs = []
    for lat in lats:
        for s, extra in enumerate((dict(double_pass=True), dict(ell_deep=[12, 4]),
                                   dict(double_pass=True, ell_deep=[16, 6], overlap=True))):
            b = torch.from_numpy(I.gaussian_source(DIMS, 60 + s).ravel()).cuda()
            jobs.append(dict(lat=lat, b=b, x=torch.empty_like(b), k=140, ell=40, **extra))

    def run(graph):
        c.tune_set("graph", int(graph))
        xs, _ = nks.sign_apply_batch(jobs, stats=False)
        torch.cuda.synchronize()
        return [to_np(x).copy() for x in xs]

    ref = run(False)
    for rep in range(3):
        got = run(True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
        y = nks.apply_op(lats[1], jobs[0]["b"])
        torch.cuda.synchronize()
        assert math.isfinite(float(torch.linalg.vector_norm(y)))
    assert c.tune_get("graph_replays") >= 2
    c.tune_set("graph", 1)


def test_double_pass_with_learned_policy_equals_single_pass():
    import paper_0912_4457_amd as nks
    nks.load_policy(ctx())
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    _pairs_of_runs([dict(lat=lat, b=I.gaussian_source(DIMS, 31).ravel(), k=1000, ell=256, tol=1e-8,
                         k_policy=nks.POLICY_LEARNED, ell_policy=nks.POLICY_LEARNED)])
