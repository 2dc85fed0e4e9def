"""Pins of the overlap operator of Sec. 2 (Eq. Dovmu) in the oracle: the
Ginsparg-Wilson relation, which follows from sgn(A)^2 = 1 alone, the unit
circle of the mu = 0 spectrum, and the nested method against the dense
operator."""
import numpy as np
import pytest

import nks_inputs as I
from oracle import dirac, overlap


def _op(mu, dims=(2, 2, 2, 2), eps=0.5, seed=11):
    return dirac.Operator(I.su3_links(dims, eps, seed), dims, 1.6, mu)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_ginsparg_wilson_relation(mu):
    # gamma5 D + D gamma5 = D gamma5 D  <=>  (gamma5 sgn(A))^2 = 1
    op = _op(mu)
    D = overlap.overlap_dense(op)
    g5 = dirac.gamma5_full(op.n // 12).toarray()
    lhs = g5 @ D + D @ g5
    rhs = D @ g5 @ D
    assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(D)
    # and the relation fails if the identity term is dropped
    S = D - np.eye(op.n)
    assert np.linalg.norm(g5 @ S + S @ g5 - S @ g5 @ S) > 1e-2 * np.linalg.norm(S)


def test_spectrum_on_the_unit_circle_at_mu0():
    # at mu = 0 gamma5 sgn(A) is unitary, so D_ov = 1 + unitary has |lambda - 1| = 1
    D = overlap.overlap_dense(_op(0.0))
    lam = np.linalg.eigvals(D)
    assert np.allclose(np.abs(lam - 1.0), 1.0, atol=1e-10)
    # and some are away from 0 and 2 (a nontrivial operator)
    assert np.ptp(lam.real) > 0.5


def test_nested_overlap_matches_dense():
    op = _op(0.0, dims=(4, 4, 4, 4), eps=0.5, seed=4401)
    x = I.gaussian_source((4, 4, 4, 4), 4402).ravel()
    ref = overlap.from_sign(op, x, overlap.nested.sign_exact_dense(op, x))
    got = overlap.overlap_apply(op, x, 400, 400)
    assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)
