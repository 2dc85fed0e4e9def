"""Graph mode of nks_sign_apply_batch: the captured launch sequence replayed
on later calls gives the eager result bit for bit, with eager work and
synchronisations between replays, and a changed operator or job table is
captured anew."""
import math

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, to_np

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)


def _jobs(nks, lats, **kw):
    """Jobs with device-resident b and x, so repeated calls see the same table."""
    import torch
    jobs = []
    for lat in lats:
        for s in range(3):
            b = torch.from_numpy(I.gaussian_source(DIMS, 50 + s).ravel()).cuda()
            jobs.append(dict(lat=lat, b=b, x=torch.empty_like(b), k=kw.get("k", 160), ell=kw.get("ell", 40),
                             tol=kw.get("tol", 1e-8),
                             k_policy=kw.get("k_policy", 0), ell_policy=kw.get("ell_policy", 0),
                             precision=kw.get("precision", "fp64")))
    return jobs


def _run(nks, jobs, graph):
    import torch
    c = jobs[0]["lat"].ctx
    c.tune_set("graph", int(graph))
    xs, _ = nks.sign_apply_batch(jobs, stats=False)
    torch.cuda.synchronize()
    return [to_np(x).copy() for x in xs]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_replays_match_eager_bitwise(precision):
    import torch
    import paper_0912_4457_amd as nks
    c = nks.Context(0)
    u = I.su3_links(DIMS, 0.5, 4401)
    lats = [nks.Lattice(c, DIMS, u, mu=0.0), nks.Lattice(c, DIMS, u, mu=0.3)]
    jobs = _jobs(nks, lats, precision=precision)
    ref = _run(nks, jobs, graph=False)
    cap0 = c.tune_get("graph_captures")
    for rep in range(3):
        got = _run(nks, jobs, graph=True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
        # eager work between replays
        y = nks.apply_op(lats[1], jobs[0]["b"])
        torch.cuda.synchronize()
        assert math.isfinite(float(torch.linalg.vector_norm(y)))
    assert c.tune_get("graph_captures") == cap0 + 1
    assert c.tune_get("graph_replays") >= 2


def test_changed_operator_is_captured_anew():
    import paper_0912_4457_amd as nks
    c = nks.Context(0)
    lat = nks.Lattice(c, DIMS, I.su3_links(DIMS, 0.5, 4401), mu=0.0)
    jobs = _jobs(nks, [lat])
    _run(nks, jobs, graph=True)
    n0 = c.tune_get("graph_captures")
    lat.set_params(1.5, 0.0)                       # new kappa: a launch argument
    got = _run(nks, jobs, graph=True)
    assert c.tune_get("graph_captures") == n0 + 1
    ref = _run(nks, jobs, graph=False)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_new_source_and_output_buffers_replay_the_graph():
    """b and x are read from the job table uploaded before each replay, so a
    call with new buffers (and new data) replays the captured graph and gives
    the eager result for the new data, bit for bit."""
    import torch
    import paper_0912_4457_amd as nks
    c = nks.Context(0)
    u = I.su3_links(DIMS, 0.5, 4401)
    lats = [nks.Lattice(c, DIMS, u, mu=0.0), nks.Lattice(c, DIMS, u, mu=0.3)]
    jobs = _jobs(nks, lats)
    _run(nks, jobs, graph=True)
    n0, r0 = c.tune_get("graph_captures"), c.tune_get("graph_replays")
    fresh = []
    for i, j in enumerate(jobs):
        b = torch.from_numpy(I.gaussian_source(DIMS, 900 + i).ravel()).cuda()
        fresh.append(dict(j, b=b, x=torch.empty_like(b)))
    got = _run(nks, fresh, graph=True)
    assert c.tune_get("graph_captures") == n0 and c.tune_get("graph_replays") == r0 + 1
    ref = _run(nks, fresh, graph=False)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_policies_in_graph_mode_match_eager():
    import paper_0912_4457_amd as nks
    from paper_0912_4457_amd import policy as P
    c = nks.Context(0)
    params = np.zeros(P.NPARAMS, np.float32)
    params[-2:] = [math.log10(250), math.log10(32)]
    nks.policy_load(c, P.pack(params, np.zeros(16), np.ones(16), np.zeros(2), np.ones(2)))
    u = I.su3_links(DIMS, 0.5, 4401)
    lats = [nks.Lattice(c, DIMS, u, mu=0.0), nks.Lattice(c, DIMS, u, mu=0.3)]
    for pol in (1, 2):
        jobs = _jobs(nks, lats, k=800, ell=200, tol=1e-8, k_policy=pol, ell_policy=pol)
        ref = _run(nks, jobs, graph=False)
        for rep in range(2):
            got = _run(nks, jobs, graph=True)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (pol, rep)
