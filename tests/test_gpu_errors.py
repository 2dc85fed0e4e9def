"""Error paths and degenerate inputs of the C ABI (each call returns an error
code before any kernel is launched, or reports a status), and an uneven
batch (lattices of different sizes, k and mu in one call) against single
calls."""
import ctypes

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, lattice, to_np

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)


def _sign_with(opts_mutator, lat=None, b=None):
    """nks_sign_apply through the C ABI with a hand-modified nks_opts."""
    import torch
    import paper_0912_4457_amd as nks
    lat = lat or lattice(DIMS, 0.5, 4401, 0.0)
    b = torch.from_numpy(I.gaussian_source(DIMS, 3).ravel()).cuda() if b is None else b
    x = torch.empty_like(b)
    o = nks.make_opts(k=60, ell=20)
    opts_mutator(o)
    ws = lat.ctx.workspace(1 << 26)
    st = nks.Stats()
    rc = nks.lib().nks_sign_apply(lat.ctx.h, lat.h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(), None,
                                  ctypes.byref(st))
    return rc, st, x


@pytest.mark.parametrize("field,value", [("k", 0), ("ell", 0), ("precision", 7), ("max_rhi_iter", 0),
                                         ("rhi_tol", 0.0), ("k_policy", 5), ("ell_policy", -1), ("size", 8)])
def test_invalid_options_are_rejected(field, value):
    rc, _, _ = _sign_with(lambda o: setattr(o, field, value))
    assert rc == 1, (field, rc)


def test_policy_without_tolerance_is_rejected():
    def m(o):
        o.k_policy, o.tol = 1, 0.0
    rc, _, _ = _sign_with(m)
    assert rc == 1


def test_size_limits_are_reported_as_unsupported():
    def big_ell(o):
        o.k, o.ell = 1200, 1100          # nested with a dense RHi above 1024
    def big_nonnested(o):
        o.k, o.ell = 1100, 2000          # non-nested RHi on H_k above 1024
    assert _sign_with(big_ell)[0] == 4
    assert _sign_with(big_nonnested)[0] == 4


def test_undersized_workspace_is_rejected():
    import torch
    import paper_0912_4457_amd as nks
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    b = torch.from_numpy(I.gaussian_source(DIMS, 3).ravel()).cuda()
    x = torch.empty_like(b)
    o = nks.make_opts(k=60, ell=20)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    rc = nks.lib().nks_sign_apply(lat.ctx.h, lat.h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.byref(o), ctypes.c_void_p(small.data_ptr()), small.numel(), None, None)
    assert rc == 2


def test_lattice_parameters_are_validated():
    import paper_0912_4457_amd as nks
    lat = nks.Lattice(ctx(), DIMS, I.su3_links(DIMS, 0.5, 4401))
    for m0, mu in ((2.5, 0.0), (0.0, 0.0), (1.6, float("nan"))):
        with pytest.raises(nks.NKSError) as e:
            lat.set_params(m0, mu)
        assert e.value.code == 1
    with pytest.raises(nks.NKSError):
        nks.Lattice(ctx(), (1, 4, 4, 4), I.unit_links((1, 4, 4, 4)))
    for key, value in (("xcd_map", 4), ("collapse", 0), ("min_waves", 2), ("no_such_key", 1)):
        with pytest.raises(nks.NKSError):
            ctx().tune_set(key, value)


def test_rhi_iteration_cap_reports_noconv():
    rc, st, x = _sign_with(lambda o: setattr(o, "max_rhi_iter", 1))
    assert rc == 0 and st.status == 6 and st.rhi_iters == 1


def test_odd_sizes_round_up_to_even():
    rc, st, _ = _sign_with(lambda o: (setattr(o, "k", 61), setattr(o, "ell", 21)))
    assert rc == 0 and st.status == 0 and st.k_used == 62 and st.ell_used == 22


def test_uneven_batch_equals_single_calls():
    import paper_0912_4457_amd as nks
    specs = [((4, 4, 4, 4), 0.0, 80), ((4, 4, 4, 6), 0.3, 60), ((6, 4, 4, 4), 0.1, 100), ((4, 4, 4, 6), 0.3, 40)]
    jobs = []
    for i, (dims, mu, k) in enumerate(specs):
        lat = lattice(dims, 0.4, 70 + len(dims) + dims[0] + dims[3], mu)
        jobs.append(dict(lat=lat, b=I.gaussian_source(dims, 90 + i).ravel(), k=k, ell=20))
    xs, sts = nks.sign_apply_batch(jobs)
    for j, x, st in zip(jobs, xs, sts):
        x1, st1 = nks.sign_apply(j["lat"], j["b"], k=j["k"], ell=j["ell"])
        assert st["status"] == 0 and st["k_used"] == st1["k_used"]
        assert np.array_equal(to_np(x), to_np(x1))
