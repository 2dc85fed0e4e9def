"""Multi-level nesting of Sec. 4.5 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Level 0 is the outer Ritz matrix T_0 = H_k (size k_0 = k, App. C step 2).
For a level i below the deepest one, sgn(T_i) e_1 is approximated in the
Krylov space K_{k_{i+1}}(T_i', e_1) with the preconditioned matrix
T_i' = (p_i T_i + (p_i T_i)^{-1}) / 2 of Eq. precond, exactly as the single
nested level of Sec. 4.1 does for H_k: (two-sided) Lanczos on T_i' (the
inverse by an LU of p_i T_i) gives the tridiagonal Ritz matrix T_{i+1} and
the basis W_i, and sgn(T_i) e_1 ~ W_i sgn(T_{i+1}) e_1 (Eq. innersign,
since sgn(T_i') = sgn(T_i) by Eq. proofprec).  At the deepest level L the
sign of T_L comes from RHi.  So the outer coefficients are

    c = W_0 W_1 ... W_{L-1} sgn(T_L) e_1,   y = |b| V_k c   (Eq. nested).

p_i follows Eq. popt with the Ritz-value extremes of T_i (the footnote of
Sec. 4.5 takes them from the previous level's spectrum the same way);
with more levels p_i tends to 1 and the preconditioning step tends to one
RHi step.  L = 1 is the nested method of Sec. 4.1.

A requested size k_{i+1} >= k_i (after rounding up to even) makes level i
exact: RHi runs on T_i itself and the recursion stops there (the rule the
single-level method uses for ell >= k), unless ``force_nested``.
"""
from __future__ import annotations

import numpy as np

from . import krylov
from .nested import TridiagLU, ritz_extremes, tridiag_matvec
from .precond import p_opt
from .signfun import rhi


def _tridiag_dense(alpha, beta, gamma):
    h = np.diag(alpha)
    if len(alpha) > 1:
        h = h + np.diag(beta, -1) + np.diag(gamma, 1)
    return h


def _level(alpha, beta, gamma, hermitian, size, p, zmax_bound=None):
    """One level: Lanczos on T' from e_1 with ``size`` steps.

    Returns (inner Krylov result, p used, z_min, z_max)."""
    k = len(alpha)
    zmin = zmax = None
    if p is None or p <= 0:
        zmin, zmax = ritz_extremes(alpha, beta, gamma, hermitian, zmax_bound)
        p = p_opt(zmin, zmax)
    p = float(p)
    lu = TridiagLU(p * beta, p * alpha, p * gamma)
    if lu.info != 0:
        raise np.linalg.LinAlgError("p T_i is singular")

    def tp(v):
        return 0.5 * (lu.solve(v, "N") + p * tridiag_matvec(beta, alpha, gamma, v))

    def tp_dag(v):
        return 0.5 * (lu.solve(v, "C") + p * tridiag_matvec(np.conj(gamma), np.conj(alpha), np.conj(beta), v))

    e1 = np.zeros(k, dtype=np.float64 if hermitian else np.complex128)
    e1[0] = 1.0
    if hermitian:
        inner = krylov.lanczos(tp, e1, size)
    else:
        inner = krylov.two_sided_lanczos(tp, tp_dag, e1, size)
    return inner, p, zmin, zmax


def multilevel_coefficients(alpha, beta, gamma, hermitian: bool, sizes, ps=None,
                            force_nested: bool = False, zmax_bound: float | None = None):
    """c ~ sgn(T_0) e_1 for the tridiagonal T_0 = H_k by ``len(sizes)`` nested
    levels; ``sizes[i]`` = k_{i+1} (rounded up to even), ``ps[i]`` = p_i
    (None or <= 0: p_opt from the Ritz values of T_i; at level 0 with z_max
    capped at ``zmax_bound``, a bound of A's spectrum, as in the one-level
    method; the deeper T_i have their own spectra).

    Returns (c, info); info holds the sizes and p of the levels that ran,
    the RHi iterations at the deepest level and a status."""
    if hermitian:
        a = np.asarray(alpha, float).real
        b = np.asarray(beta, float).real
        g = b
    else:
        a = np.asarray(alpha, complex)
        b = np.asarray(beta, complex)
        g = np.asarray(gamma, complex)
    sizes = [krylov.even_up(int(s)) for s in sizes]
    ps = list(ps) if ps is not None else [None] * len(sizes)
    info = dict(sizes=[len(a)], p=[], z_min=[], z_max=[], status="ok")
    bases = []
    for i, size in enumerate(sizes):
        k = len(a)
        if size >= k and not force_nested:
            break                                       # level i is exact: RHi on T_i
        inner, p, zmin, zmax = _level(a, b, g, hermitian, min(size, k), ps[i], zmax_bound if i == 0 else None)
        info["p"].append(p)
        info["z_min"].append(zmin)
        info["z_max"].append(zmax)
        if inner.status == "breakdown":
            info["status"] = "breakdown"
        bases.append(inner.V)
        a, b, g = inner.alpha, inner.beta, inner.gamma
        if hermitian:
            a, b, g = np.real(a), np.real(b), np.real(b)
        info["sizes"].append(len(a))
    s, it, ok = rhi(_tridiag_dense(a, b, g))
    info["rhi_iters"] = it
    if not ok:
        info["status"] = "noconv"
    c = s[:, 0]
    for W in reversed(bases):                           # c = W_0 ... W_{L-1} sgn(T_L) e_1
        c = W @ c
    info["levels"] = len(bases)
    return c, info


def sign_apply(op, x, k: int, sizes, ps=None, force_nested: bool = False):
    """y ~ sgn(A) x with the outer basis of size k and nested levels ``sizes``."""
    x = np.asarray(x, dtype=np.complex128)
    xf = x.ravel()
    if op.hermitian:
        kr = krylov.lanczos(op.matvec, xf, k)
    else:
        kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, xf, k)
    if kr.status == "zero":
        return np.zeros_like(x), dict(sizes=[0], p=[], status="ok", levels=0)
    c, info = multilevel_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, sizes, ps, force_nested,
                                      zmax_bound=op.norm_bound)
    info["k"] = kr.k_used
    if kr.status == "breakdown":
        info["status"] = "breakdown"
    y = kr.bnorm * (kr.V @ c)
    info["alpha"], info["beta"], info["gamma"] = kr.alpha, kr.beta, kr.gamma
    info["c"] = c
    return y.reshape(x.shape), info
