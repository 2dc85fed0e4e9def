"""Tolerance-driven choice of ell and k (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not in the paper: it fixes k (Sec. 4.2) and reads ell_opt off the curves of
Figs. 7-9.  The plain policy written here (and, separately, on the GPU):

* ell-doubling.  Start at ell_0 = 16.  Compute c_ell and c_2ell (the inner
  Krylov space of size 2 ell extends the one of size ell).  Accept c_2ell when
  ||c_2ell - c_ell|| <= (tol/10) ||c_2ell||, otherwise double again.  Once
  2 ell reaches the cap (min(ell_max, k)) the non-nested RHi on H_k is used.
* k-checkpoints.  Every dk = 100 outer iterations run the nested step (with
  ell-doubling) on H_k and stop when the coefficient change
  ||c^(k) - [c^(k-dk); 0]||_w <= (tol/4) ||c^(k)||_w, where ||d||_w^2 =
  sum_j |d_j|^2 ||v_j||^2 (the basis norms; all 1 in the Hermitian case, where
  this is exactly the change of y / |b|).
"""
from __future__ import annotations

import numpy as np

from . import krylov
from .nested import nested_coefficients

ELL0 = 16
DK = 100


def ell_doubling(alpha, beta, gamma, hermitian: bool, tol: float, ell_max: int | None = None,
                 p: float | None = None, zmax_bound: float | None = None):
    """Returns (c, info) with info['ell'] (0 if non-nested) and info['inner_delta'];
    ``zmax_bound`` caps z_max of the p_opt estimate (``nested.ritz_extremes``)."""
    k = len(alpha)
    cap = k if ell_max is None else min(int(ell_max), k)
    ell = ELL0
    if ell >= cap:
        c, info = nested_coefficients(alpha, beta, gamma, hermitian, k)
        info["inner_delta"] = 0.0
        return c, info
    c_prev, info = nested_coefficients(alpha, beta, gamma, hermitian, ell, p, zmax_bound=zmax_bound)
    while True:
        ell2 = 2 * ell
        if ell2 >= cap:
            if cap >= k:
                c, info = nested_coefficients(alpha, beta, gamma, hermitian, k)
            else:
                c, info = nested_coefficients(alpha, beta, gamma, hermitian, cap, p, zmax_bound=zmax_bound)
            info["inner_delta"] = float(np.linalg.norm(c - c_prev) / np.linalg.norm(c))
            return c, info
        c, info = nested_coefficients(alpha, beta, gamma, hermitian, ell2, p, zmax_bound=zmax_bound)
        delta = float(np.linalg.norm(c - c_prev) / np.linalg.norm(c))
        if delta <= tol / 10:
            info["inner_delta"] = delta
            return c, info
        ell, c_prev = ell2, c


def weighted_norm(d, vnorm):
    return float(np.sqrt(np.sum(np.abs(d) ** 2 * vnorm[:len(d)] ** 2)))


def sign_apply_policy(op, x, tol: float, k_max: int, ell_max: int | None = None, dk: int = DK):
    """y ~ sgn(A) x with k by checkpoints and ell by doubling; returns (y, info)."""
    x = np.asarray(x, dtype=np.complex128)
    xf = x.ravel()
    if op.hermitian:
        kr = krylov.lanczos(op.matvec, xf, k_max)
    else:
        kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, xf, k_max)
    if kr.status == "zero":
        return np.zeros_like(x), {"k": 0, "ell": 0, "outer_delta": 0.0, "converged": True}
    vnorm = np.linalg.norm(kr.V, axis=0)
    c_prev = None
    k = dk
    converged = False
    while True:
        kk = min(k, kr.k_used)
        sl = slice(0, kk)
        c, info = ell_doubling(kr.alpha[sl], kr.beta[:kk - 1], kr.gamma[:kk - 1], op.hermitian, tol, ell_max,
                               zmax_bound=op.norm_bound)
        if c_prev is not None:
            d = c.copy()
            d[:len(c_prev)] -= c_prev
            delta = weighted_norm(d, vnorm) / weighted_norm(c, vnorm)
            info["outer_delta"] = delta
            if delta <= tol / 4:
                converged = True
                break
        if kk >= kr.k_used:
            break
        c_prev = c
        k += dk
    info["k"] = kk
    info["converged"] = converged
    y = kr.bnorm * (kr.V[:, :kk] @ c)
    return y.reshape(x.shape), info
