"""GPU parity of the Wilson stencil A = gamma5 D_w(mu) (and A^dagger) against
the oracle's explicit CSR matrix, from tiny to the full 8^4 / 10^4 sizes."""
import numpy as np
import pytest

import nks_inputs as I
from gpu_common import lattice, operator, rel, to_np

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (3, 4, 5, 6), (8, 8, 8, 8), (10, 10, 10, 10)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("dagger", [False, True])
def test_stencil_fp64_matches_csr(dims, mu, dagger):
    import paper_0912_4457_amd as nks
    lat = lattice(dims, 0.5, 77, mu)
    op = operator(dims, 0.5, 77, mu)
    v = I.gaussian_source(dims, 5).ravel()
    y = to_np(nks.apply_op(lat, v, dagger=dagger))
    ref = (op.AH if dagger else op.A) @ v
    assert rel(y, ref) <= 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (10, 10, 10, 10)])
@pytest.mark.parametrize("mu", [0.0, 0.2])
def test_stencil_fp32_matches_csr(dims, mu):
    import paper_0912_4457_amd as nks
    lat = lattice(dims, 0.35, 78, mu)
    op = operator(dims, 0.35, 78, mu)
    v = I.gaussian_source(dims, 6).ravel()
    y = to_np(nks.apply_op(lat, v, precision="mixed"))
    assert rel(y, op.A @ v) <= 1e-6


def test_stencil_adjoint_identity_on_gpu():
    import paper_0912_4457_amd as nks
    dims = (4, 6, 4, 6)
    lat = lattice(dims, 0.6, 79, 0.3)
    v = I.gaussian_source(dims, 7).ravel()
    w = I.gaussian_source(dims, 8).ravel()
    av = to_np(nks.apply_op(lat, v))
    ahw = to_np(nks.apply_op(lat, w, dagger=True))
    assert abs(np.vdot(w, av) - np.vdot(ahw, v)) <= 1e-13 * abs(np.vdot(w, av))


def test_stencil_point_source_sparsity():
    # A e_x touches only x and its 8 neighbours
    import paper_0912_4457_amd as nks
    dims = (4, 4, 4, 4)
    lat = lattice(dims, 0.5, 77, 0.0)
    b = I.point_source(dims, 1, 2, site=5).ravel()
    y = to_np(nks.apply_op(lat, b)).reshape(-1, 12)
    nz = np.nonzero(np.abs(y).sum(axis=1))[0]
    assert len(nz) == 9


@pytest.mark.parametrize("kind", ["gaussian", "u3_phase"])
def test_stencil_with_general_links(kind):
    # the stencil takes the links as given: no SU(3) structure is assumed
    import paper_0912_4457_amd as nks
    from oracle import dirac
    from gpu_common import ctx, M0
    dims = (4, 4, 4, 4)
    if kind == "gaussian":
        rng = np.random.default_rng(82)
        u = (rng.standard_normal(dims + (4, 3, 3)) + 1j * rng.standard_normal(dims + (4, 3, 3))) / 3
    else:
        u = I.su3_links(dims, 0.5, 83) * np.exp(0.4j)      # unitary, det = e^{1.2 i}
    lat = nks.Lattice(ctx(), dims, u, m0=M0, mu=0.1)
    op = dirac.Operator(u, dims, M0, 0.1)
    v = I.gaussian_source(dims, 10).ravel()
    y = to_np(nks.apply_op(lat, v))
    assert rel(y, op.A @ v) <= 1e-14
    lat.close()
