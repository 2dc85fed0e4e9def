"""Explicit sparse Wilson-Dirac operator at chemical potential (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the definition of D_w(mu) in Sec. 2 literally:

    D_w(mu) = 1 - kappa sum_{i=1..3} (T_i^+ + T_i^-)
                - kappa (e^{mu} T_4^+ + e^{-mu} T_4^-),
    (T_nu^{+-})_{yx} = (1 +- gamma_nu) U_{x,+-nu} delta_{y, x +- nu_hat},
    U_{x,-nu} = U_{x-nu_hat,+nu}^dagger,   kappa = 1/(8 + 2 m_w),

and A = gamma5 D_w(mu) (the argument of sgn in Eq. Dovmu).  Read per output
row y: T^+ brings psi(y - nu_hat) with (1 + gamma_nu) U_{y-nu_hat,+nu}, and
T^- brings psi(y + nu_hat) with (1 - gamma_nu) U_{y,+nu}^dagger.

Readings where the paper is silent: periodic boundaries in all four
directions; Euclidean gamma matrices in the chiral basis
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]],
so that gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def pauli():
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    return s1, s2, s3


def gamma_matrices():
    """(gamma_1..gamma_4, gamma_5) in the chiral basis, Euclidean, Hermitian."""
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    gs = [np.block([[z, -1j * s], [1j * s, z]]) for s in pauli()]
    gs.append(np.block([[z, one], [one, z]]))
    g5 = gs[0] @ gs[1] @ gs[2] @ gs[3]
    return gs, g5


def kappa_from_m0(m0: float) -> float:
    """kappa = 1/(8 + 2 m_w) with m_w = -m0, m_w in (-2, 0)."""
    mw = -float(m0)
    if not (-2.0 < mw < 0.0):
        raise ValueError("m_w = -m0 must lie in (-2, 0)")
    return 1.0 / (8.0 + 2.0 * mw)


def _site_grid(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel(), t.ravel()


def _site_index(x, y, z, t, dims):
    lx, ly, lz, lt = dims
    return (x % lx) + lx * ((y % ly) + ly * ((z % lz) + lz * (t % lt)))


def neighbour(dims, nu: int, sign: int) -> np.ndarray:
    """Index of site x + sign*nu_hat for every site x (periodic)."""
    x, y, z, t = _site_grid(dims)
    c = [x, y, z, t]
    c[nu] = c[nu] + sign
    return _site_index(*c, dims)


def wilson_csr(links: np.ndarray, dims, kappa: float, mu: float) -> sp.csr_matrix:
    """D_w(mu) as a CSR matrix of size 12V x 12V (index 12*site+3*spin+colour)."""
    dims = tuple(int(d) for d in dims)
    V = dims[0] * dims[1] * dims[2] * dims[3]
    u = links.reshape(V, 4, 3, 3)
    gs, _ = gamma_matrices()
    one4 = np.eye(4, dtype=np.complex128)
    rows, cols, vals = [], [], []
    sites = np.arange(V)

    def add_blocks(row_sites, col_sites, blocks):
        # blocks: (V, 12, 12)
        r = 12 * row_sites[:, None, None] + np.arange(12)[None, :, None]
        c = 12 * col_sites[:, None, None] + np.arange(12)[None, None, :]
        r, c = np.broadcast_arrays(r, c)
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(blocks.ravel())

    # identity
    add_blocks(sites, sites, np.broadcast_to(np.eye(12, dtype=np.complex128), (V, 12, 12)))
    for nu in range(4):
        cp = np.exp(mu) if nu == 3 else 1.0   # coefficient of T_nu^+
        cm = np.exp(-mu) if nu == 3 else 1.0  # coefficient of T_nu^-
        back = neighbour(dims, nu, -1)  # y - nu_hat
        fwd = neighbour(dims, nu, +1)   # y + nu_hat
        # T^+: row y, column y - nu_hat, block (1 + gamma_nu) x U_{y-nu_hat,+nu}
        ub = u[back, nu]
        blk = np.einsum("ij,sab->siajb", one4 + gs[nu], ub).reshape(V, 12, 12)
        add_blocks(sites, back, -kappa * cp * blk)
        # T^-: row y, column y + nu_hat, block (1 - gamma_nu) x U_{y,+nu}^dagger
        uf = np.conj(np.swapaxes(u[:, nu], -1, -2))
        blk = np.einsum("ij,sab->siajb", one4 - gs[nu], uf).reshape(V, 12, 12)
        add_blocks(sites, fwd, -kappa * cm * blk)
    m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(12 * V, 12 * V)).tocsr()
    m.sum_duplicates()
    m.eliminate_zeros()
    return m


def gamma5_full(V: int) -> sp.csr_matrix:
    _, g5 = gamma_matrices()
    return sp.kron(sp.identity(V, format="csr"), sp.kron(sp.csr_matrix(g5),
                   sp.identity(3, format="csr"))).tocsr()


def hermitian_wilson_csr(links, dims, m0: float, mu: float) -> sp.csr_matrix:
    """A = gamma5 D_w(mu) with kappa = 1/(8 - 2 m0); Hermitian iff mu = 0."""
    V = int(np.prod(dims))
    d = wilson_csr(links, dims, kappa_from_m0(m0), mu)
    return (gamma5_full(V) @ d).tocsr()


def norm_bound(m0: float, mu: float) -> float:
    """Upper bound of ||A|| = ||D_w(mu)|| (Sec. 2), hence of every |lambda| of A.

    D_w = 1 - kappa sum_nu (c_+ (1 - gamma_nu) U S_+ + c_- (1 + gamma_nu) U^dag S_-)
    with shifts S_+-, c_+- = 1 in space and e^{+-mu} in time.  (1 -+ gamma_nu)/2
    are complementary orthogonal projectors and U S_+- are unitary, so each
    direction's hop term has norm <= 2 kappa sqrt(c_+^2 + c_-^2): 2 sqrt(2) kappa
    in space, 2 sqrt(2 cosh 2mu) kappa in time."""
    kappa = kappa_from_m0(m0)
    return 1.0 + kappa * (6.0 * np.sqrt(2.0) + 2.0 * np.sqrt(2.0 * np.cosh(2.0 * mu)))


class Operator:
    """A = gamma5 D_w(mu) with both A v and A^dagger v (CSR conjugate transpose)."""

    def __init__(self, links, dims, m0: float, mu: float):
        self.dims = tuple(int(d) for d in dims)
        self.m0 = float(m0)
        self.mu = float(mu)
        self.norm_bound = norm_bound(self.m0, self.mu)
        self.A = hermitian_wilson_csr(links, self.dims, m0, mu)
        self.AH = self.A.conj().T.tocsr()
        self.n = self.A.shape[0]
        self.hermitian = (mu == 0.0)

    def matvec(self, v):
        return self.A @ v

    def rmatvec(self, v):
        return self.AH @ v

    def dense(self):
        return self.A.toarray()
