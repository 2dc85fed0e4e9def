"""Deflated sign application (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

App. C step 1 and the first sum of step 6: with m eigenpairs (lambda_i, r_i)
of A and left eigenvectors l_i (l_i^dagger r_j = delta_ij),

    x_m = x - sum_i <l_i, x> r_i,
    sgn(A) x = sgn(A) x_m + sum_i sgn(lambda_i) <l_i, x> r_i,

and the Krylov-Ritz method runs on x_m only, whose spectral content has no
weight on the deflated eigenvalues.  sgn(lambda) = sgn(Re lambda) (Eq. sgnz).
"""
from __future__ import annotations

import numpy as np

from . import nested


def project(x, r, l):
    """(x_m, d) with d_i = <l_i, x> and x_m = x - sum_i d_i r_i; r, l: (m, n)."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    d = np.conj(l) @ x
    return x - d @ r, d


def sign_apply_deflated(op, x, k: int, ell: int, r, l, lam, p: float | None = None):
    """sgn(A) x with the nested method on the deflated source."""
    xm, d = project(x, r, l)
    if np.linalg.norm(xm) == 0.0:
        y, info = np.zeros_like(xm), {"k": 0}
    else:
        y, info = nested.sign_apply(op, xm, k, ell, p=p)
    return np.asarray(y).ravel() + (np.sign(np.real(lam)) * d) @ r, info


def eigenpairs_smallest(op, m: int):
    """The m eigenpairs of smallest |lambda| from the dense A, with left
    eigenvectors normalised to l_i^dagger r_i = 1 (for tests on small lattices)."""
    a = op.dense()
    if op.hermitian:
        w, v = np.linalg.eigh(a)
        idx = np.argsort(np.abs(w))[:m]
        r = v[:, idx].T.copy()
        return w[idx].astype(np.complex128), r, r.copy()
    import scipy.linalg as sla
    w, vl, vr = sla.eig(a, left=True, right=True)
    idx = np.argsort(np.abs(w))[:m]
    r = vr[:, idx].T.copy()
    l = vl[:, idx].T.copy()
    for i in range(m):
        s = np.vdot(l[i], r[i])
        l[i] = l[i] / np.conj(s)
    return w[idx], r, l
