"""nks_sign_apply_noalloc (the workspace is the library's static per-GPU array)
against nks_sign_apply with a caller workspace: the same kernels on the same
inputs, so the same bits; two calls in a row, the second on a smaller input
than the first, and a job too large for the array is refused."""
import ctypes

import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, lattice, to_np

pytestmark = pytest.mark.gpu

CASES = (((6, 6, 6, 6), 0.4, 6401, 0.3, 6402, 200, 40),    # two-sided, 15552 x 200 basis
         ((4, 4, 4, 4), 0.5, 4401, 0.0, 4402, 100, 20))    # Hermitian, smaller


def test_noalloc_matches_sign_apply_on_two_calls():
    import paper_0912_4457_amd as nks
    c = ctx()
    for dims, eps, seed, mu, src, k, ell in CASES:
        lat = lattice(dims, eps, seed, mu)
        b = I.gaussian_source(dims, src).ravel()
        x_ref, st_ref = nks.sign_apply(lat, b, k=k, ell=ell)
        x, st = nks.sign_apply_noalloc(lat, b, k=k, ell=ell)
        assert st["status"] == 0 and st_ref["status"] == 0
        assert (st["k_used"], st["ell_used"], st["rhi_iters"]) == (st_ref["k_used"], st_ref["ell_used"],
                                                                    st_ref["rhi_iters"])
        assert np.array_equal(to_np(x), to_np(x_ref)), (dims, mu)
        assert np.linalg.norm(to_np(x)) > 0


def test_noalloc_without_stats_and_too_large_job():
    import paper_0912_4457_amd as nks
    dims, eps, seed, mu, src, k, ell = CASES[1]
    lat = lattice(dims, eps, seed, mu)
    b = I.gaussian_source(dims, src).ravel()
    x_ref, _ = nks.sign_apply(lat, b, k=k, ell=ell)
    x, st = nks.sign_apply_noalloc(lat, b, k=k, ell=ell, stats=False)
    import torch
    torch.cuda.synchronize()
    assert st is None and np.array_equal(to_np(x), to_np(x_ref))
    # 4^4 with k = 4000 needs 3072 * 4000 * 16 bytes of basis: more than the static array
    with pytest.raises(nks.NKSError) as e:
        nks.sign_apply_noalloc(lat, b, k=4000, ell=20)
    assert e.value.code == 2 and "NKS_NOALLOC_BYTES" in e.value.args[0]
    # the double-pass mode of the same job fits
    x2, st2 = nks.sign_apply_noalloc(lat, b, k=k, ell=ell, double_pass=True)
    assert st2["status"] == 0 and np.array_equal(to_np(x2), to_np(x_ref))


def test_noalloc_rejects_null_arguments():
    import paper_0912_4457_amd as nks
    c = ctx()
    o = nks.make_opts(k=20, ell=10)
    assert nks.lib().nks_sign_apply_noalloc(c.h, None, None, None, ctypes.byref(o), None, None) != 0
