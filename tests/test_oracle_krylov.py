"""Pins of the oracle's Lanczos (App. A) and two-sided Lanczos (App. B)."""
import numpy as np
import pytest

import nks_inputs as I
from oracle import closedform, dirac, krylov, nested

M0 = 1.6


def _op(mu, dims=(3, 3, 3, 3), eps=0.5, seed=21):
    return dirac.Operator(I.su3_links(dims, eps, seed), dims, M0, mu)


def test_lanczos_invariants():
    op = _op(0.0)
    b = I.gaussian_source(op.dims, 1).ravel()
    kr = krylov.lanczos(op.matvec, b, 24)
    V = kr.V
    assert kr.k_used == 24
    assert np.abs(V.conj().T @ V - np.eye(24)).max() < 1e-12
    T = V.conj().T @ (op.A @ V)
    assert np.abs(T - kr.H()).max() < 1e-12
    assert np.isrealobj(kr.alpha) and np.all(kr.beta > 0)
    assert np.allclose(V[:, 0], b / np.linalg.norm(b))


def test_two_sided_invariants():
    op = _op(0.3)
    b = I.gaussian_source(op.dims, 2).ravel()
    kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, 20, keep_left=True)
    V, W = kr.V, kr.W
    assert np.abs(W.conj().T @ V - np.eye(20)).max() < 1e-10
    H = W.conj().T @ (op.A @ V)
    assert np.abs(H - kr.H()).max() < 1e-10
    # principal branch beta = sqrt(delta), gamma = conj(delta)/beta
    assert np.all(kr.beta.real >= 0)
    H = kr.H()
    assert np.abs(np.triu(H, 2)).max() == 0 and np.abs(np.tril(H, -2)).max() == 0


def test_even_rounding():
    op = _op(0.0)
    kr = krylov.lanczos(op.matvec, I.gaussian_source(op.dims, 3).ravel(), 15)
    assert kr.k_used == 16


def test_lucky_breakdown_free_field_gives_exact_result():
    # U = 1 on 2^4: few distinct eigenvalues, so the Krylov space is invariant early
    dims = (2, 2, 2, 2)
    for mu in (0.0, 0.3):
        op = dirac.Operator(I.unit_links(dims), dims, M0, mu)
        b = I.gaussian_source(dims, 4)
        y, info = nested.sign_apply(op, b, 60, 60)
        assert info["k"] < 60
        ref = closedform.free_field_sign_apply(b, dims, M0, mu)
        assert nested.rel_err(y, ref) < 1e-10


def test_serious_breakdown_detected():
    # first row (a, 0, 1), first column (a, 1, 0), x = e_1: r = e_2, l = e_3, r^dagger l = 0
    a = 0.7
    A = np.array([[a, 0, 1], [1, 2.0, 0.5], [0, 0.3, -1.0]], dtype=complex)
    x = np.array([1, 0, 0], dtype=complex)
    kr = krylov.two_sided_lanczos(lambda v: A @ v, lambda v: A.conj().T @ v, x, 4)
    assert kr.status == "breakdown" and kr.k_used == 1


def test_zero_source():
    op = _op(0.0)
    y, info = nested.sign_apply(op, np.zeros(op.n, complex), 20, 10)
    assert np.all(y == 0)
    op = _op(0.3)
    y, info = nested.sign_apply(op, np.zeros(op.n, complex), 20, 10)
    assert np.all(y == 0)


def test_two_sided_reduces_to_lanczos_for_hermitian():
    op = _op(0.0)
    b = I.gaussian_source(op.dims, 5).ravel()
    k1 = krylov.lanczos(op.matvec, b, 30)
    k2 = krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, 30)
    assert np.allclose(k1.alpha, k2.alpha.real, atol=1e-11)
    assert np.allclose(k1.beta, k2.beta.real, atol=1e-11)
    assert np.allclose(k2.beta, k2.gamma, atol=1e-11)
