"""Seeded synthetic inputs: gauge links, gauge transformations and source vectors.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds no arithmetic of the sign-function method itself: it only draws random
numbers and shapes them into SU(3) matrices and spinor fields.

Conventions (all arrays are numpy, complex128):

* ``dims = (Lx, Ly, Lz, Lt)``; the site index is ``x + Lx*(y + Ly*(z + Lz*t))``,
  i.e. a C-order flattening of an array of shape ``(Lt, Lz, Ly, Lx)``.
* Links: shape ``(Lt, Lz, Ly, Lx, 4, 3, 3)``; ``links[..., nu, :, :]`` is the
  forward link U_{x,+nu} with nu = 0, 1, 2, 3 for the x, y, z, t directions.
  The link transports a colour vector from site x to site x + nu_hat (the
  Wilson operator of Sec. 2 uses U_{x,+nu} on the hop that lands on x + nu_hat).
* Spinor fields: shape ``(V, 4, 3)`` (site, spin, colour); flattened, the
  component index is ``12*site + 3*spin + colour``.

The synthetic links stand in for the paper's lattice QCD configurations
(which are not available): U = exp(i*eps*sum_a theta_a lambda_a) with
theta_a ~ N(0, 1) per link and Gell-Mann matrices lambda_a.  Small eps gives
smooth (near-free) fields, larger eps rougher ones.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "gell_mann",
    "su3_links",
    "unit_links",
    "random_su3_field",
    "pure_gauge_links",
    "gaussian_source",
    "point_source",
    "ones_source",
    "config",
]


def volume(dims) -> int:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or min(dims) < 1:
        raise ValueError(f"dims must be four positive extents, got {dims}")
    return dims[0] * dims[1] * dims[2] * dims[3]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, normalised tr(l_a l_b) = 2 delta_ab."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1], l[1, 1, 0] = -1j, 1j
    l[2, 0, 0], l[2, 1, 1] = 1, -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2], l[4, 2, 0] = -1j, 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2], l[6, 2, 1] = -1j, 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def _expi_hermitian(x: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*X) for a stack of Hermitian 3x3 matrices X (via eigh)."""
    w, v = np.linalg.eigh(x)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def su3_links(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i eps sum_a theta_a lambda_a), theta ~ N(0,1).

    theta is drawn as one array of shape (Lt, Lz, Ly, Lx, 4, 8) in C order from
    ``numpy.random.default_rng(seed)``.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    volume(dims)
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal((lt, lz, ly, lx, 4, 8))
    x = np.einsum("...a,aij->...ij", theta, gell_mann())
    return _expi_hermitian(x, float(eps))


def unit_links(dims) -> np.ndarray:
    lx, ly, lz, lt = (int(d) for d in dims)
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def random_su3_field(dims, seed: int) -> np.ndarray:
    """Haar-random SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3).

    QR of a complex Gaussian matrix with the phases of R's diagonal moved
    into Q gives a Haar-random U(3) matrix; dividing by a cube root of its
    determinant puts it in SU(3).
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((lt, lz, ly, lx, 3, 3))
         + 1j * rng.standard_normal((lt, lz, ly, lx, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


def pure_gauge_links(g: np.ndarray) -> np.ndarray:
    """Links of a pure gauge: U_{x,+nu} = g_{x+nu_hat} g_x^dagger (periodic).

    With this transport convention the Wilson operator on these links is the
    free operator conjugated by the block-diagonal field g.
    """
    lt, lz, ly, lx = g.shape[:4]
    u = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    gd = np.conj(np.swapaxes(g, -1, -2))
    # array axes (t, z, y, x) <-> directions (3, 2, 1, 0)
    for nu, axis in ((0, 3), (1, 2), (2, 1), (3, 0)):
        g_fwd = np.roll(g, -1, axis=axis)  # g at x + nu_hat
        u[..., nu, :, :] = g_fwd @ gd
    return u


def gaussian_source(dims, seed: int) -> np.ndarray:
    """b = (N(0,1) + i N(0,1)) / sqrt(2) per component, shape (V, 4, 3)."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((v, 4, 3))
    im = rng.standard_normal((v, 4, 3))
    return (re + 1j * im) / np.sqrt(2)


def point_source(dims, spin: int, colour: int, site: int = 0) -> np.ndarray:
    v = volume(dims)
    b = np.zeros((v, 4, 3), dtype=np.complex128)
    b[site, spin, colour] = 1.0
    return b


def ones_source(dims) -> np.ndarray:
    """The test vector x = (1, ..., 1) used for the error estimates of Sec. 3."""
    return np.ones((volume(dims), 4, 3), dtype=np.complex128)


# Synthetic workloads.  m0 is the positive mass parameter: the Wilson mass is
# m_w = -m0 and kappa = 1 / (8 + 2 m_w).
_CONFIGS = {
    # 4^4 Hermitian, Lanczos k=200, nested ell=50, one Gaussian source
    "hermitian_4x4": dict(dims=(4, 4, 4, 4), eps=0.5, link_seed=4401, mu=0.0,
                          m0=1.6, src_seed=4402, k=200, ell=50),
    # 8^4 at mu=0.3, two-sided Lanczos k=800, nested ell~150
    "nonhermitian_8x4": dict(dims=(8, 8, 8, 8), eps=0.4, link_seed=8401, mu=0.3,
                             m0=1.6, src_seed=8402, k=800, ell=150),
    # 10^4, 12 spin-colour point sources at the origin, mu in {0, 0.2}
    "point12_10x4_mu0": dict(dims=(10, 10, 10, 10), eps=0.35, link_seed=10401,
                             mu=0.0, m0=1.6, tol=1e-8),
    "point12_10x4_mu02": dict(dims=(10, 10, 10, 10), eps=0.35, link_seed=10401,
                              mu=0.2, m0=1.6, tol=1e-8),
}


def sketch_rows(n: int, rows, seed: int) -> np.ndarray:
    """Rows ``rows`` (an iterable of row indices) of a seeded complex Gaussian
    sketch matrix S of shape (total rows, n) with E|S_ij|^2 = 1; each row is
    drawn from its own generator, so any subset of rows is reproducible on
    its own.  For a vector e, |S e|^2 / (number of rows) estimates |e|^2 (a
    chi-square with 2 * rows degrees of freedom: with 256 rows the estimate of
    |e| has a relative spread of about 3 %)."""
    out = []
    for i in rows:
        rng = np.random.default_rng([seed, int(i)])
        out.append((rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(0.5))
    return np.array(out)


def config(name: str) -> dict:
    """A copy of one named synthetic workload description."""
    return dict(_CONFIGS[name])
