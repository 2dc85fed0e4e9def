"""Exact sgn(A)b for free and pure-gauge links, in momentum space (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Derived from the definition of D_w(mu) in Sec. 2 and Eq. sgnz.  With U = 1 a
plane wave psi(y) = e^{i p.y} phi satisfies psi(y -+ nu_hat) = e^{-+ i p_nu} psi(y),
so the hop terms give, per direction,

    c^+ e^{-i p}(1 + gamma) + c^- e^{i p}(1 - gamma) = 2 cos q - 2 i sin q gamma,

with q_nu = p_nu (spatial) and q_4 = p_4 + i mu (from e^{+-mu}).  Hence

    D~(p) = a + i sum_nu b_nu gamma_nu,  a = 1 - 2 kappa sum_nu cos q_nu,
    b_nu = 2 kappa sin q_nu,

and H~ = gamma5 D~ squares to (a^2 + sum_nu b_nu^2) times the identity (even
for complex a, b), so sgn(H~) = H~ / sqrt(a^2 + sum b^2) with the principal
root of Eq. sgnz.  A pure gauge U_{x,nu} = g_{x+nu_hat} g_x^dagger gives
A[U] = G A[1] G^dagger with G = diag(g_x), so sgn(A[U]) b = G sgn(A[1]) G^dagger b.

Both functions work at any lattice size (the 10^4 lattice included).
"""
from __future__ import annotations

import numpy as np

from .dirac import gamma_matrices, kappa_from_m0


def _momentum_symbol(dims, kappa, mu):
    """H~(p) = gamma5 D~(p) for all momenta; shape (Lt, Lz, Ly, Lx, 4, 4)."""
    lx, ly, lz, lt = dims
    gs, g5 = gamma_matrices()
    # numpy's fftn over axes (t, z, y, x): momentum p = 2 pi n / L per axis
    pt = 2 * np.pi * np.fft.fftfreq(lt) * 1.0
    pz = 2 * np.pi * np.fft.fftfreq(lz)
    py = 2 * np.pi * np.fft.fftfreq(ly)
    px = 2 * np.pi * np.fft.fftfreq(lx)
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    q = [PX.astype(np.complex128), PY.astype(np.complex128),
         PZ.astype(np.complex128), PT + 1j * mu]
    a = 1.0 - 2.0 * kappa * sum(np.cos(qn) for qn in q)
    b = [2.0 * kappa * np.sin(qn) for qn in q]
    d = a[..., None, None] * np.eye(4)
    for nu in range(4):
        d = d + 1j * b[nu][..., None, None] * gs[nu]
    h = g5 @ d
    s2 = a * a + sum(bn * bn for bn in b)
    return h, s2


def free_field_spectrum(dims, m0: float, mu: float):
    """Eigenvalues +-sqrt(a^2 + sum b^2) of A[U=1] (each with multiplicity)."""
    _, s2 = _momentum_symbol(tuple(dims), kappa_from_m0(m0), mu)
    r = np.sqrt(s2.astype(np.complex128)).ravel()
    return np.concatenate([r, -r])


def free_field_sign_apply(b: np.ndarray, dims, m0: float, mu: float) -> np.ndarray:
    """sgn(gamma5 D_w(mu)[U=1]) b for b of shape (V, 4, 3) (or flat 12V)."""
    dims = tuple(int(d) for d in dims)
    lx, ly, lz, lt = dims
    shape_in = b.shape
    bb = np.asarray(b, dtype=np.complex128).reshape(lt, lz, ly, lx, 4, 3)
    h, s2 = _momentum_symbol(dims, kappa_from_m0(m0), mu)
    sg = h / np.sqrt(s2.astype(np.complex128))[..., None, None]
    bt = np.fft.fftn(bb, axes=(0, 1, 2, 3))
    yt = np.einsum("...ij,...jc->...ic", sg, bt)
    y = np.fft.ifftn(yt, axes=(0, 1, 2, 3))
    return y.reshape(shape_in)


def free_field_apply(b: np.ndarray, dims, m0: float, mu: float) -> np.ndarray:
    """A[U=1] b = gamma5 D_w(mu) b computed in momentum space."""
    dims = tuple(int(d) for d in dims)
    lx, ly, lz, lt = dims
    shape_in = b.shape
    bb = np.asarray(b, dtype=np.complex128).reshape(lt, lz, ly, lx, 4, 3)
    h, _ = _momentum_symbol(dims, kappa_from_m0(m0), mu)
    bt = np.fft.fftn(bb, axes=(0, 1, 2, 3))
    y = np.fft.ifftn(np.einsum("...ij,...jc->...ic", h, bt), axes=(0, 1, 2, 3))
    return y.reshape(shape_in)


def pure_gauge_sign_apply(b: np.ndarray, g: np.ndarray, dims, m0: float,
                          mu: float) -> np.ndarray:
    """sgn(A[U]) b for U_{x,nu} = g_{x+nu_hat} g_x^dagger (g: (Lt,Lz,Ly,Lx,3,3))."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    gv = g.reshape(V, 3, 3)
    bb = np.asarray(b, dtype=np.complex128).reshape(V, 4, 3)
    gdb = np.einsum("sba,sib->sia", gv.conj(), bb)        # G^dagger b
    y = free_field_sign_apply(gdb, dims, m0, mu).reshape(V, 4, 3)
    return np.einsum("sab,sib->sia", gv, y).reshape(b.shape)  # G (...)
