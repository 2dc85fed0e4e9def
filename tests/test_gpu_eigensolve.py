"""GPU eigensolver for the deflation eigenpairs (nks_lattice_eigensolve,
Hermitian A): eigenvalues and eigenvectors against the oracle's dense
eigendecomposition, residuals recomputed with the oracle's operator, the
installed pairs in a deflated sign application against the oracle's
deflated method, and the error paths."""
import numpy as np
import pytest

import nks_inputs as I
from gpu_common import ctx, lattice, operator, rel, to_np

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)


def test_eigenpairs_match_dense_eigendecomposition():
    from oracle import deflation
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    op = operator(DIMS, 0.5, 4401, 0.0)
    m = 8
    try:
        lam, res, it = lat.compute_deflation(m, tol=1e-10)
        r, _ = lat.deflation_vectors()
        r = to_np(r)
    finally:
        lat.set_deflation(None, [])
    lam_ref, r_ref, _ = deflation.eigenpairs_smallest(op, m)
    print(f"{it} iterations, worst residual {res.max():.1e}")
    assert np.all(res <= 1e-10) and it >= 1
    assert np.all(np.diff(np.abs(lam)) >= 0)
    order = np.argsort(np.abs(lam_ref))
    assert np.allclose(lam, np.real(lam_ref[order]), rtol=0, atol=1e-9)
    A = op.dense()
    for i in range(m):
        x = r[i]
        assert abs(np.linalg.norm(x) - 1) <= 1e-12
        # residual recomputed with the oracle's operator
        assert np.linalg.norm(A @ x - lam[i] * x) <= 2e-10
        # the same eigenvector up to a phase (the eigenvalues are simple)
        ov = abs(np.vdot(r_ref[order[i]], x)) / np.linalg.norm(r_ref[order[i]])
        assert np.sqrt(max(0.0, 1 - ov * ov)) <= 1e-6
    G = r.conj() @ r.T
    assert np.abs(G - np.eye(m)).max() <= 1e-12


def test_computed_pairs_deflate_like_the_oracle():
    import paper_0912_4457_amd as nks
    from oracle import deflation, nested
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    op = operator(DIMS, 0.5, 4401, 0.0)
    b = I.gaussian_source(DIMS, 4402).ravel()
    m = 12
    lam_ref, r_ref, l_ref = deflation.eigenpairs_smallest(op, m)
    xm, _ = deflation.project(b, r_ref, l_ref)
    _, info = nested.sign_apply(op, xm, 100, 30)
    ref, _ = deflation.sign_apply_deflated(op, b, 100, 30, r_ref, l_ref, lam_ref, p=info["p"])
    try:
        lat.compute_deflation(m, tol=1e-11)
        x, st = nks.sign_apply(lat, b, k=100, ell=30, p=info["p"], deflate=True)
    finally:
        lat.set_deflation(None, [])
    assert st["status"] == 0
    assert rel(to_np(x), ref) <= 1e-8


@pytest.mark.parametrize("dims,eps,seed,m", [((8, 8, 8, 8), 0.4, 8401, 12), ((10, 10, 10, 10), 0.35, 10401, 8)])
def test_eigensolve_residuals_with_the_oracle_operator(dims, eps, seed, m):
    lat = lattice(dims, eps, seed, 0.0)
    op = operator(dims, eps, seed, 0.0)
    try:
        lam, res, it = lat.compute_deflation(m, max_iter=400, tol=1e-10)
        r, _ = lat.deflation_vectors()
        r = to_np(r)
    finally:
        lat.set_deflation(None, [])
    print(f"{dims}: {it} iterations, |lambda| {np.abs(lam).min():.4f}..{np.abs(lam).max():.4f}")
    for i in range(m):
        assert np.linalg.norm(op.matvec(r[i]) - lam[i] * r[i]) <= 2e-10
    assert np.abs(r.conj() @ r.T - np.eye(m)).max() <= 1e-12


def test_eigensolve_errors():
    import paper_0912_4457_amd as nks
    lat2 = lattice(DIMS, 0.5, 4401, 0.3)
    with pytest.raises(nks.NKSError) as e:
        lat2.compute_deflation(4)
    assert e.value.code == 4
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    for m in (0, 65):
        with pytest.raises(nks.NKSError) as e:
            lat.compute_deflation(m)
        assert e.value.code == 1
    with pytest.raises(nks.NKSError) as e:      # too few iterations: no convergence, nothing installed
        lat.compute_deflation(4, max_iter=1, tol=1e-12)
    assert e.value.code == 6
    r, _ = lat.deflation_vectors()
    assert r.shape[0] == 0


def test_sign_of_computed_eigenvectors():
    # sgn(A) r = sgn(lambda) r for the eigenpairs the eigensolver returns (Eq. fAdef)
    import paper_0912_4457_amd as nks
    lat = lattice(DIMS, 0.5, 4401, 0.0)
    try:
        lam, res, it = lat.compute_deflation(4, tol=1e-11)
        r, _ = lat.deflation_vectors()
    finally:
        lat.set_deflation(None, [])
    for i in range(4):
        x, st = nks.sign_apply(lat, r[i].clone(), k=300, ell=80)
        assert st["status"] == 0
        assert rel(to_np(x), np.sign(lam[i]) * to_np(r[i])) <= 1e-9
