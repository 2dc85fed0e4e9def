"""Pins of the oracle's Wilson-Dirac operator (definition of D_w(mu), Sec. 2).

Each check compares the explicit CSR matrix with something derived
independently: the momentum-space symbol (free field), the gauge-covariance
identity (pure gauge / random gauge transformation), the adjoint identity
A(mu)^dagger = A(-mu), or the Clifford algebra.
"""
import numpy as np
import pytest

import nks_inputs as I
from oracle import closedform, dirac

M0 = 1.6
DIMS_SET = [(2, 2, 2, 2), (3, 3, 3, 3), (2, 3, 4, 5)]


def test_gamma_clifford_and_gamma5():
    gs, g5 = dirac.gamma_matrices()
    for a in range(4):
        assert np.allclose(gs[a], gs[a].conj().T)
        for b in range(4):
            assert np.allclose(gs[a] @ gs[b] + gs[b] @ gs[a], 2 * np.eye(4) * (a == b))
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


def test_kappa_reading():
    # kappa = 1/(8 + 2 m_w) with m_w = -m0 in (-2, 0)
    assert dirac.kappa_from_m0(1.6) == pytest.approx(1 / 4.8)
    with pytest.raises(ValueError):
        dirac.kappa_from_m0(2.5)
    with pytest.raises(ValueError):
        dirac.kappa_from_m0(0.0)


@pytest.mark.parametrize("dims", DIMS_SET)
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_matches_momentum_symbol(dims, mu):
    op = dirac.Operator(I.unit_links(dims), dims, M0, mu)
    b = I.gaussian_source(dims, 11)
    y_csr = op.matvec(b.ravel())
    y_ft = closedform.free_field_apply(b, dims, M0, mu).ravel()
    assert np.linalg.norm(y_csr - y_ft) <= 1e-13 * np.linalg.norm(y_ft)


@pytest.mark.parametrize("mu", [0.0, 0.25])
def test_adjoint_identity(mu):
    dims = (2, 3, 4, 3)
    u = I.su3_links(dims, 0.7, 3)
    a = dirac.hermitian_wilson_csr(u, dims, M0, mu)
    am = dirac.hermitian_wilson_csr(u, dims, M0, -mu)
    # A(mu)^dagger = gamma5 D_w(-mu) = A(-mu)
    assert abs(a.conj().T - am).max() < 1e-15
    if mu == 0.0:
        assert abs(a - a.conj().T).max() < 1e-15
    else:
        assert abs(a - a.conj().T).max() > 1e-3


def test_gauge_covariance():
    dims = (3, 2, 2, 4)
    V = int(np.prod(dims))
    u = I.su3_links(dims, 0.6, 7)
    g = I.random_su3_field(dims, 8)
    # U^g_{x,nu} = g_{x+nu} U_{x,nu} g_x^dagger  (transport x -> x + nu_hat)
    ug = np.empty_like(u)
    gd = np.conj(np.swapaxes(g, -1, -2))
    for nu, axis in ((0, 3), (1, 2), (2, 1), (3, 0)):
        ug[..., nu, :, :] = np.roll(g, -1, axis=axis) @ u[..., nu, :, :] @ gd
    for mu in (0.0, 0.3):
        a = dirac.hermitian_wilson_csr(u, dims, M0, mu)
        ag = dirac.hermitian_wilson_csr(ug, dims, M0, mu)
        b = I.gaussian_source(dims, 9)
        gv = g.reshape(V, 3, 3)
        gdb = np.einsum("sba,sib->sia", gv.conj(), b)
        lhs = ag @ b.ravel()
        rhs = np.einsum("sab,sib->sia", gv, (a @ gdb.ravel()).reshape(V, 4, 3)).ravel()
        assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_sparsity_and_links_unitary():
    dims = (4, 4, 4, 4)
    u = I.su3_links(dims, 0.5, 4401)
    uu = np.einsum("...ab,...cb->...ac", u, u.conj())
    assert np.allclose(uu, np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.det(u), 1.0, atol=1e-12)
    a = dirac.hermitian_wilson_csr(u, dims, M0, 0.3)
    nnz_per_row = np.diff(a.indptr)
    # diagonal + 8 hops x (2 spin x 3 colour)
    assert nnz_per_row.max() == 49


def test_plane_wave_eigenvector_free_field():
    dims = (4, 4, 4, 4)
    lx, ly, lz, lt = dims
    op = dirac.Operator(I.unit_links(dims), dims, M0, 0.0)
    n = np.array([1, 0, 2, 3])
    p = 2 * np.pi * n / np.array(dims)
    t, z, y, x = np.meshgrid(*[np.arange(L) for L in (lt, lz, ly, lx)], indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).ravel()
    h, _ = closedform._momentum_symbol(dims, dirac.kappa_from_m0(M0), 0.0)
    hp = h[n[3] % lt, n[2] % lz, n[1] % ly, n[0] % lx]
    w, vecs = np.linalg.eigh(hp)
    spin = vecs[:, 0]
    psi = (phase[:, None, None] * spin[None, :, None] * np.array([1, 0, 0])[None, None, :]).ravel()
    assert np.linalg.norm(op.matvec(psi) - w[0] * psi) < 1e-12 * np.linalg.norm(psi)


@pytest.mark.parametrize("kind", ["su3", "unit"])
@pytest.mark.parametrize("mu", [0.0, 0.2, 0.5])
def test_norm_bound_holds(kind, mu):
    """|lambda| <= ||A||_2 <= dirac.norm_bound(m0, mu) (Sec. 2 operator), and the
    bound is within 30 % of ||A||_2 on the free field (so it can cap a
    spectrum estimate without cutting into it by much)."""
    dims = (4, 2, 2, 4)                  # even extents: the free field reaches momentum pi
    u = I.su3_links(dims, 0.6, 77) if kind == "su3" else I.unit_links(dims)
    op = dirac.Operator(u, dims, 1.6, mu)
    a = op.dense()
    smax = np.linalg.norm(a, 2)
    bound = dirac.norm_bound(1.6, mu)
    assert op.norm_bound == bound
    assert np.abs(np.linalg.eigvals(a)).max() <= smax * (1 + 1e-12)
    assert smax <= bound
    if kind == "unit" and mu == 0.0:
        assert smax >= 0.7 * bound
