"""Pins of the deflated sign application (App. C steps 1 and 6) in the
oracle: deflating every eigenpair gives the spectral sign exactly, the
deflated source has no weight on the deflated left eigenvectors, and
deflating the smallest eigenvalues speeds up the Krylov-Ritz convergence."""
import numpy as np
import pytest

import nks_inputs as I
from oracle import deflation, dirac, nested


def _op(mu, dims=(2, 2, 2, 2), eps=0.5, seed=11):
    return dirac.Operator(I.su3_links(dims, eps, seed), dims, 1.6, mu)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_deflation_is_the_spectral_sign(mu):
    op = _op(mu)
    lam, r, l = deflation.eigenpairs_smallest(op, op.n)
    x = I.gaussian_source((2, 2, 2, 2), 5).ravel()
    y, _ = deflation.sign_apply_deflated(op, x, 20, 8, r, l, lam)
    ref = nested.sign_exact_dense(op, x)
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_deflated_source_is_orthogonal_to_left_vectors(mu):
    op = _op(mu, dims=(3, 3, 3, 3))
    lam, r, l = deflation.eigenpairs_smallest(op, 12)
    assert np.allclose(np.conj(l) @ r.T, np.eye(12), atol=1e-10)
    xm, d = deflation.project(I.gaussian_source((3, 3, 3, 3), 6).ravel(), r, l)
    assert np.abs(np.conj(l) @ xm).max() <= 1e-10 * np.linalg.norm(xm)


def test_deflation_speeds_up_convergence():
    op = _op(0.0, dims=(4, 4, 4, 4), eps=0.5, seed=4401)
    x = I.gaussian_source((4, 4, 4, 4), 4402).ravel()
    ref = nested.sign_exact_dense(op, x)
    lam, r, l = deflation.eigenpairs_smallest(op, 32)
    y0, _ = nested.sign_apply(op, x, 120, 120)
    y1, _ = deflation.sign_apply_deflated(op, x, 120, 120, r, l, lam)
    e0 = np.linalg.norm(y0.ravel() - ref.ravel()) / np.linalg.norm(ref)
    e1 = np.linalg.norm(y1 - ref.ravel()) / np.linalg.norm(ref)
    assert e1 < 0.1 * e0


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_eigenpairs_satisfy_both_eigen_equations(mu):
    # A r_i = lambda_i r_i and l_i^dagger A = lambda_i l_i^dagger, ascending |lambda|;
    # real spectrum for the Hermitian A (mu = 0), a complex one otherwise
    op = _op(mu, dims=(3, 3, 3, 3))
    lam, r, l = deflation.eigenpairs_smallest(op, 10)
    A = op.dense()
    for i in range(10):
        assert np.linalg.norm(A @ r[i] - lam[i] * r[i]) <= 1e-12 * np.linalg.norm(r[i])
        assert np.linalg.norm(l[i].conj() @ A - lam[i] * l[i].conj()) <= 1e-12 * np.linalg.norm(l[i])
    assert np.all(np.diff(np.abs(lam)) >= 0)
    if mu == 0.0:
        assert np.abs(lam.imag).max() <= 1e-14
    else:
        assert np.abs(lam.imag).max() >= 1e-4
