"""Full-size parity: the 10^4 workload of the benchmark (12 spin-colour point
sources at mu = 0 and mu = 0.2 in one batched call, the benchmark's k, ell
and launch configuration) against the oracle's converged results stored in
tests/golden/point12_10x4.json (written by make_point12_10x4.py, which calls
only the oracle).  For every source the full-vector error estimated from
the reference's 256-row Gaussian sketch (tests/golden/point12_10x4_sketch.npz,
make_sketch_10x4.py), 256 sampled entries plus the full norm, and the complete
vectors of four of the sources."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "point12_10x4.json")


def _gold():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_file_is_converged():
    g = _gold()
    assert len(g["cases"]) == 24
    for c in g["cases"]:
        # the reference's own accuracy (change from a shorter basis) is far below the tested tolerance
        assert c["change_from_k_check"] <= 1e-9, c
        assert len(c["idx"]) >= 128


def _run(precision):
    import torch
    import bench
    import paper_0912_4457_amd as nks
    from gpu_common import ctx
    c = ctx()
    lats, jobs = bench.make_jobs(nks, torch, c, precision)
    xs, sts = nks.sign_apply_batch(jobs, stats=True)
    torch.cuda.synchronize()
    return jobs, xs, sts, lats


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_point12_10x4_matches_oracle(precision, tol):
    import bench
    g = _gold()
    jobs, xs, sts, lats = _run(precision)
    # complete vectors of four sources (tests/golden/point4_full_10x4.npz,
    # make_full_10x4.py: the same converged oracle reference)
    full = bench.full_golden()
    assert full is not None and len(full["mu"]) == 4
    assert np.all(full["change_from_k_check"] <= 1e-9)
    ferrs = bench.errors_vs_full(jobs, xs, full)
    assert len(ferrs) == 4
    for mu, spin, colour, e in ferrs:
        print(f"{precision}: mu={mu} spin={spin} colour={colour}: full-vector rel err {e:.2e}")
        assert e <= tol, (mu, spin, colour, e)
    # every source: the sketch estimate (3 % spread, so 0.85 tol bounds the
    # true error by tol with a margin of five spreads) and the sampled entries
    sk = bench.errors_vs_sketch(jobs, xs, bench.sketch_golden())
    assert sk is not None and len(sk) == 24
    for (mu, spin, colour, e) in ferrs:
        est = next(s for j, s in zip(jobs, sk) if (j["mu"], j["spin"], j["colour"]) == (mu, spin, colour))
        assert abs(est - e) <= 0.15 * e, (mu, spin, colour, est, e)
    errs = bench.sampled_errors(jobs, xs, g)
    for j, x, st, e, es in zip(jobs, xs, sts, errs, sk):
        case = next(c for c in g["cases"]
                    if c["mu"] == j["mu"] and c["spin"] == j["spin"] and c["colour"] == j["colour"])
        assert st["status"] == 0 and st["k_used"] == bench.K_MU[j["mu"]], st
        nrm = float(np.linalg.norm(x.cpu().numpy()))
        assert abs(nrm - case["norm"]) <= tol * case["norm"], (j["mu"], j["spin"], j["colour"], nrm, case["norm"])
        assert e <= tol, (j["mu"], j["spin"], j["colour"], e)
        assert es <= 0.85 * tol, (j["mu"], j["spin"], j["colour"], es)
    print(f"{precision}: max full-vector rel err (sketch estimate) {max(sk):.2e}, max sampled {max(errs):.2e} "
          f"over {len(errs)} sources")
