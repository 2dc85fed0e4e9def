"""Scalar and dense matrix sign functions (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``sgn``        -- Eq. sgnz: sgn(z) = z / sqrt(z^2) with the square-root cut
                    on the negative real axis, i.e. sgn(Re z).
* ``sign_eig``   -- Eq. fAdef: f(A) = U f(Lambda) U^{-1} (eigh when Hermitian).
* ``rhi``        -- Eq. Roberts: S_0 = H, S_{n+1} = (S_n + S_n^{-1}) / 2.

RHi stopping rule (the paper only says it converges within 7-10 iterations
to machine precision): stop when the relative Frobenius change
||S_{n+1} - S_n||_F / ||S_{n+1}||_F is <= 1e-14; once it is <= 1e-8 the
quadratic convergence makes the next step the last one; give up after
``maxit`` iterations.
"""
from __future__ import annotations

import numpy as np

RHI_TOL = 1e-14
RHI_NEAR = 1e-8
RHI_MAXIT = 50


def sgn(z):
    """sgn(z) = z / sqrt(z^2) (principal root); equals sign(Re z) off the cut."""
    z = np.asarray(z, dtype=np.complex128)
    return z / np.sqrt(z * z)


def sign_eig(a: np.ndarray, hermitian: bool | None = None) -> np.ndarray:
    """Spectral definition of the matrix sign function."""
    a = np.asarray(a)
    if hermitian is None:
        hermitian = np.allclose(a, a.conj().T, atol=0, rtol=1e-13)
    if hermitian:
        w, u = np.linalg.eigh(a)
        s = np.sign(w)
        return (u * s) @ u.conj().T
    w, u = np.linalg.eig(a)
    s = np.sign(w.real)
    return np.linalg.solve(u.T, (u * s).T).T  # U diag(s) U^{-1}


def rhi(h: np.ndarray, tol: float = RHI_TOL, near: float = RHI_NEAR,
        maxit: int = RHI_MAXIT):
    """Roberts-Higham iteration; returns (S, iterations, converged)."""
    s = np.array(h, dtype=np.result_type(h, np.float64), copy=True)
    last = False
    for it in range(1, maxit + 1):
        s_new = 0.5 * (s + np.linalg.inv(s))
        change = np.linalg.norm(s_new - s) / np.linalg.norm(s_new)
        s = s_new
        if change <= tol or last:
            return s, it, True
        if change <= near:
            last = True
    return s, maxit, False
