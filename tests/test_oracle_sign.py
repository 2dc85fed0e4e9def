"""Pins of the oracle's sign functions (Eqs. sgnz, fAdef, Roberts) and of the
closed forms sgn(A)b for free and pure-gauge links."""
import numpy as np
import pytest
import scipy.linalg as sla

import nks_inputs as I
from oracle import closedform, dirac, nested, signfun

M0 = 1.6


def test_scalar_sgn():
    rng = np.random.default_rng(0)
    z = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    s = signfun.sgn(z)
    assert np.allclose(s * s, 1)
    assert np.allclose(s, np.sign(z.real))
    x = rng.standard_normal(50)
    assert np.allclose(signfun.sgn(x), np.sign(x))


@pytest.mark.parametrize("herm", [True, False])
def test_sign_eig_and_rhi_match_scipy_signm(herm):
    rng = np.random.default_rng(1)
    n = 40
    m = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if herm:
        m = m + m.conj().T
    else:
        # eigenvalues well away from the imaginary axis
        w = np.concatenate([rng.uniform(0.5, 3, n // 2), -rng.uniform(0.5, 3, n - n // 2)])
        w = w + 0.3j * rng.standard_normal(n)
        q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        m = q @ np.diag(w) @ np.linalg.inv(q)
    ref = sla.signm(m)
    s_eig = signfun.sign_eig(m, hermitian=herm)
    s_rhi, it, ok = signfun.rhi(m)
    assert ok
    assert np.linalg.norm(s_eig - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(s_rhi - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(s_rhi @ s_rhi - np.eye(n)) < 1e-9


def test_rhi_iteration_count_on_lattice_ritz_matrix():
    # Sec. 3: 7 to 10 iterations for QCD-like Ritz matrices
    dims = (3, 3, 3, 3)
    op = dirac.Operator(I.su3_links(dims, 0.5, 5), dims, M0, 0.0)
    from oracle import krylov
    kr = krylov.lanczos(op.matvec, I.gaussian_source(dims, 6).ravel(), 120)
    _, it, ok = signfun.rhi(kr.H().real)
    assert ok and 6 <= it <= 12


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 3, 3, 3), (2, 2, 3, 4)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_closed_form_vs_dense(dims, mu):
    op = dirac.Operator(I.unit_links(dims), dims, M0, mu)
    b = I.gaussian_source(dims, 2)
    y_dense = nested.sign_exact_dense(op, b)
    y_cf = closedform.free_field_sign_apply(b, dims, M0, mu)
    assert nested.rel_err(y_cf, y_dense) < 1e-12


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_pure_gauge_closed_form_vs_dense(mu):
    dims = (2, 3, 2, 3)
    g = I.random_su3_field(dims, 3)
    op = dirac.Operator(I.pure_gauge_links(g), dims, M0, mu)
    b = I.gaussian_source(dims, 4)
    y_dense = nested.sign_exact_dense(op, b)
    y_cf = closedform.pure_gauge_sign_apply(b, g, dims, M0, mu)
    assert nested.rel_err(y_cf, y_dense) < 1e-12


def test_free_field_spectrum_bounds():
    # mu = 0, m_w = -1.6: z_min = 1/6 (one momentum component pi), z_max = 8/3
    z = np.abs(closedform.free_field_spectrum((4, 4, 4, 4), M0, 0.0))
    assert z.min() == pytest.approx(1 / 6, rel=1e-12)
    assert z.max() == pytest.approx(8 / 3, rel=1e-12)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_dense_sign_square_and_eigenvectors(mu):
    dims = (2, 2, 2, 3)
    op = dirac.Operator(I.su3_links(dims, 0.6, 12), dims, M0, mu)
    a = op.dense()
    s = signfun.sign_eig(a, hermitian=(mu == 0.0))
    assert np.linalg.norm(s @ s - np.eye(a.shape[0])) < 1e-10
    w, v = np.linalg.eig(a)
    for i in range(0, len(w), 17):
        assert np.linalg.norm(s @ v[:, i] - np.sign(w[i].real) * v[:, i]) < 1e-9
    # and sgn commutes with A
    assert np.linalg.norm(s @ a - a @ s) < 1e-10 * np.linalg.norm(a)
