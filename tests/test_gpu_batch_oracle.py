"""Batched, graph-replayed calls against the oracle directly (not only against
eager or single calls): the uneven batch of the benchmark (64 point sources
over 6^4, 8^4 and 10^4 lattices at mu in {0, 0.1, 0.3}, tolerances 1e-6 and
1e-8, l-doubling and k-checkpoint policies, Sec. 4.3) replayed from its
captured graph; for a subset of its jobs the oracle runs the nested method at
the (k, ell, p) that the policies chose for that job."""
import numpy as np
import pytest

import nks_inputs as I
from gpu_common import M0, ctx, rel, rounding_tolerance, to_np

pytestmark = pytest.mark.gpu

EPS = 0.35
LATS = (((6, 6, 6, 6), 6601), ((8, 8, 8, 8), 8801), ((10, 10, 10, 10), 10401))
MUS = (0.0, 0.1, 0.3)


def _batch(nks, c):
    import torch
    rng = np.random.default_rng(64)
    lats, links = [], {}
    for dims, seed in LATS:
        links[dims] = I.su3_links(dims, EPS, seed)
        for mu in MUS:
            lats.append(nks.Lattice(c, dims, links[dims], m0=M0, mu=mu))
    jobs, src = [], []
    for i in range(64):
        lat = lats[i % len(lats)]
        spin, colour, site = int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(lat.V))
        b = I.point_source(lat.dims, spin, colour, site).ravel()
        tb = torch.from_numpy(b).cuda()
        jobs.append(dict(lat=lat, b=tb, x=torch.empty_like(tb), k=1400, ell=256,
                         tol=float(rng.choice([1e-6, 1e-8])), precision="fp64", k_policy=1, ell_policy=1))
        src.append(b)
    return lats, links, jobs, src


def test_uneven_batch_graph_replays_match_oracle():
    import torch
    import paper_0912_4457_amd as nks
    from oracle import dirac, nested
    c = ctx()
    lats, links, jobs, src = _batch(nks, c)
    try:
        c.tune_set("graph", 0)
        _, sts = nks.sign_apply_batch(jobs, stats=True)          # the policies' choices per job
        torch.cuda.synchronize()
        c.tune_set("graph", 1)
        rep0 = c.tune_get("graph_replays")
        outs = []
        for _ in range(3):
            xs, _ = nks.sign_apply_batch(jobs, stats=False)
            torch.cuda.synchronize()
            outs.append([to_np(x).copy() for x in xs])
            nks.apply_op(lats[0], jobs[0]["b"])                  # eager work between replays
            torch.cuda.synchronize()
        assert c.tune_get("graph_replays") >= rep0 + 2
        # the 6^4 jobs at each mu and the first 8^4 Hermitian one
        subset = [i for i in range(64) if i % 9 in (0, 1, 2)][:3] + [3]
        for i in subset:
            lat, st = jobs[i]["lat"], sts[i]
            assert st["status"] == 0
            k, ell, p = int(st["k_used"]), int(st["ell_used"]), float(st["p_used"])
            op = dirac.Operator(links[lat.dims], lat.dims, M0, lat.mu)
            y_ref, _ = nested.sign_apply(op, src[i], k, ell, p=p)
            tol, resp = rounding_tolerance(lambda v: nested.sign_apply(op, v, k, ell, p=p)[0], src[i],
                                           lat.mu == 0.0, draws=2)
            for rep, out in enumerate(outs):
                err = rel(out[i], y_ref)
                assert err <= tol, (i, rep, err, tol)
            print(f"job {i}: {lat.dims} mu={lat.mu} tol={jobs[i]['tol']:g} -> k={k} ell={ell} p={p:.4f}: replayed "
                  f"result vs oracle {err:.2e}, tolerance {tol:.1e} (oracle's rounding response {resp:.1e})")
    finally:
        c.tune_set("graph", 1)
        for lat in lats:
            lat.close()
