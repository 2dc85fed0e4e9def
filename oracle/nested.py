"""The nested Krylov-Ritz approximation to sgn(A) x (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows App. C, steps 2-6, without deflation (m = 0):

2. (two-sided) Lanczos on A and x -> V_k, H_k              (``krylov``)
3. LU of p H_k with LAPACK ?gttrf                          (``TridiagLU``)
4. (two-sided) Lanczos on H_k' = (p H_k + (p H_k)^{-1})/2 from e_1^{(k)}:
   (a) (p H_k)^{-1} v by ?gttrs, (b) + p H_k v (tridiagonal multiply-add);
   for H_k'^dagger the solve uses trans='C' and the product H_k^dagger
5. RHi on H_ell -> sgn(H_ell)                             (``signfun.rhi``)
6. sgn(A) x ~ |x| V_k V_ell sgn(H_ell) e_1^{(ell)}          (Eq. nested)

Steps 3-5 are in real arithmetic when A is Hermitian.  The non-nested method
(Eqs. non-nested and non-nested-oblique) runs RHi on H_k itself.  p defaults
to p_opt = (z_min z_max)^{-1/2} (Eq. popt) from the exact Ritz values of H_k
(the paper takes them from A's spectrum; both only set the efficiency).
The error estimate of Sec. 3 is eps = |sgn(sgn(x)) - x| / (2|x|).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack

from . import krylov
from .precond import p_opt
from .signfun import RHI_MAXIT, rhi, sign_eig


class TridiagLU:
    """LU with partial pivoting of a tridiagonal matrix (LAPACK ?gttrf/?gttrs).

    ``sub``, ``diag``, ``sup`` are the sub-, main and super-diagonals.
    """

    def __init__(self, sub, diag, sup):
        diag = np.asarray(diag)
        self.complex = np.iscomplexobj(diag) or np.iscomplexobj(sub) or np.iscomplexobj(sup)
        dt = np.complex128 if self.complex else np.float64
        f = lapack.zgttrf if self.complex else lapack.dgttrf
        self.n = diag.size
        if self.n == 1:
            self.dl = np.zeros(0, dt); self.d = diag.astype(dt); self.du = np.zeros(0, dt)
            self.du2 = np.zeros(0, dt); self.ipiv = np.ones(1, np.int32)
            self.info = 0 if diag[0] != 0 else 1
            return
        self.dl, self.d, self.du, self.du2, self.ipiv, self.info = f(
            np.asarray(sub, dt), diag.astype(dt), np.asarray(sup, dt))

    def solve(self, b, trans: str = "N"):
        b = np.asarray(b)
        if self.complex:
            b = b.astype(np.complex128)
        if self.n == 1:
            d = self.d[0]
            return b / (np.conj(d) if trans == "C" else d)
        f = lapack.zgttrs if self.complex else lapack.dgttrs
        x, info = f(self.dl, self.d, self.du, self.du2, self.ipiv,
                    b.reshape(-1, 1), trans=trans)
        if info != 0:
            raise np.linalg.LinAlgError(f"gttrs info={info}")
        return x.ravel()


def tridiag_matvec(sub, diag, sup, v):
    """H v for H with H(i,i-1) = sub[i-1], H(i,i) = diag[i], H(i,i+1) = sup[i]."""
    y = diag * v
    y[1:] += sub * v[:-1]
    y[:-1] += sup * v[1:]
    return y


def ritz_extremes(alpha, beta, gamma, hermitian: bool, zmax_bound: float | None = None):
    """(z_min, z_max) of the Ritz values of H_k, the spectrum estimate behind
    p_opt of Sec. 4.1 (Eq. popt).

    Eq. popt wants the extremes of A's spectrum.  With ``zmax_bound`` (a bound
    of |lambda| over A's spectrum, ``dirac.norm_bound``) z_max is capped
    there: a larger |theta| cannot belong to A.  Hermitian Ritz values never
    exceed it; a two-sided H_k without reorthogonalisation can hold a
    spurious one far outside A's spectrum, which would mistune p.

    z_max = max |theta|.  Hermitian: z_min is the second smallest |theta|.
    The Ritz values of a Krylov space are the zeros of the Lanczos
    polynomial, and between two of them lies at least one eigenvalue of A,
    so the spectral gap of the indefinite A around 0 holds at most one Ritz
    value; that one can sit anywhere in the gap (near 0 for some sources)
    and says nothing about A's smallest |lambda|.  The second smallest
    |theta| lies outside the gap.  Two-sided: the same rule, without the
    interlacing theorem behind it (a non-normal H_k has none); a single
    Ritz value near the origin is seen there too."""
    if hermitian:
        if len(alpha) == 1:
            w = np.asarray(alpha, float)
        else:
            w = sla.eigh_tridiagonal(np.asarray(alpha, float), np.asarray(beta, float),
                                     eigvals_only=True)
        z = np.sort(np.abs(w))
    else:
        k = len(alpha)
        h = np.diag(np.asarray(alpha, complex))
        if k > 1:
            h += np.diag(np.asarray(beta, complex), -1) + np.diag(np.asarray(gamma, complex), 1)
        z = np.sort(np.abs(np.linalg.eigvals(h)))
    zmax = float(z[-1])
    if zmax_bound is not None:
        zmax = min(zmax, float(zmax_bound))
    return float(z[1] if z.size > 1 else z[0]), zmax


class NestedInfo(dict):
    pass


def nested_coefficients(alpha, beta, gamma, hermitian: bool, ell: int, p: float | None = None,
                        precondition: bool = True, force_nested: bool = False,
                        zmax_bound: float | None = None):
    """Steps 3-5: c ~ sgn(H_k) e_1^{(k)} from the tridiagonal H_k.

    Returns (c, info).  ``ell`` is rounded up to even; ``ell >= k`` runs the
    non-nested RHi on H_k unless ``force_nested``.  ``precondition=False``
    uses the plain inner space K_ell(H_k, e_1) of Sec. 4.1 (for tests).
    ``zmax_bound`` caps z_max of the p_opt estimate (``ritz_extremes``).
    """
    k = len(alpha)
    ell = krylov.even_up(ell)
    info = NestedInfo(k=k, ell=ell, p=None, z_min=None, z_max=None, rhi_iters=0,
                      status="ok", nested=True)
    if hermitian:
        alpha = np.asarray(alpha, float).real
        beta = np.asarray(beta, float).real
        gamma = beta
    else:
        alpha = np.asarray(alpha, complex)
        beta = np.asarray(beta, complex)
        gamma = np.asarray(gamma, complex)
    if ell >= k and not force_nested:
        h = np.diag(alpha)
        if k > 1:
            h = h + np.diag(beta, -1) + np.diag(gamma, 1)
        s, it, ok = rhi(h)
        info.update(nested=False, ell=k, rhi_iters=it, status="ok" if ok else "noconv")
        return s[:, 0], info
    ell = min(ell, k)
    e1 = np.zeros(k, dtype=np.float64 if hermitian else np.complex128)
    e1[0] = 1.0
    if precondition:
        if p is None:
            zmin, zmax = ritz_extremes(alpha, beta, gamma, hermitian, zmax_bound)
            info.update(z_min=zmin, z_max=zmax)
            p = p_opt(zmin, zmax)
        p = float(p)
        info["p"] = p
        lu = TridiagLU(p * beta, p * alpha, p * gamma)          # step 3
        if lu.info != 0:
            info["status"] = "singular"
            return np.full(k, np.nan), info

        def hp(v):                                              # step 4 (a)+(b)
            return 0.5 * (lu.solve(v, "N") + p * tridiag_matvec(beta, alpha, gamma, v))

        def hp_dag(v):
            return 0.5 * (lu.solve(v, "C")
                          + p * tridiag_matvec(np.conj(gamma), np.conj(alpha), np.conj(beta), v))
    else:
        def hp(v):
            return tridiag_matvec(beta, alpha, gamma, v)

        def hp_dag(v):
            return tridiag_matvec(np.conj(gamma), np.conj(alpha), np.conj(beta), v)

    if hermitian:
        inner = krylov.lanczos(hp, e1, ell)
    else:
        inner = krylov.two_sided_lanczos(hp, hp_dag, e1, ell)
    info["ell"] = inner.k_used
    info["inner_status"] = inner.status
    s, it, ok = rhi(inner.H())                                 # step 5
    info["rhi_iters"] = it
    if not ok:
        info["status"] = "noconv"
    c = inner.V @ s[:, 0]                                       # V_ell sgn(H_ell) e_1
    return c, info


def sign_apply(op, x, k: int, ell: int, p: float | None = None,
               precondition: bool = True, force_nested: bool = False):
    """Nested approximation y ~ sgn(A) x (Eq. nested); returns (y, info)."""
    x = np.asarray(x, dtype=np.complex128)
    shape = x.shape
    xf = x.ravel()
    if op.hermitian:
        kr = krylov.lanczos(op.matvec, xf, k)
    else:
        kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, xf, k)
    if kr.status == "zero":
        info = NestedInfo(k=0, ell=0, status="ok", p=None, rhi_iters=0, nested=False)
        return np.zeros(shape, np.complex128), info
    c, info = nested_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, ell, p,
                                  precondition, force_nested, zmax_bound=op.norm_bound)
    info["k"] = kr.k_used
    info["outer_status"] = kr.status
    if kr.status == "breakdown":
        info["status"] = "breakdown"
    y = kr.bnorm * (kr.V @ c)                                   # step 6
    info["c"] = c
    info["alpha"], info["beta"], info["gamma"] = kr.alpha, kr.beta, kr.gamma
    return y.reshape(shape), info


def nonnested_sign_apply(op, x, k: int, use_eig: bool = False):
    """Non-nested Krylov-Ritz y = |x| V_k sgn(H_k) e_1 (RHi or eig on H_k)."""
    x = np.asarray(x, dtype=np.complex128)
    xf = x.ravel()
    if op.hermitian:
        kr = krylov.lanczos(op.matvec, xf, k)
    else:
        kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, xf, k)
    if kr.status == "zero":
        return np.zeros_like(x), {"k": 0}
    h = kr.H()
    if op.hermitian:
        h = h.real
    if use_eig:
        s = sign_eig(h, hermitian=op.hermitian)
        it = 0
    else:
        s, it, _ = rhi(h, maxit=RHI_MAXIT)
    y = kr.bnorm * (kr.V @ s[:, 0])
    return y.reshape(x.shape), {"k": kr.k_used, "rhi_iters": it, "status": kr.status}


def sign_exact_dense(op, x):
    """y* = sgn(A) x from the spectral definition (Eq. fAdef), dense."""
    s = sign_eig(op.dense(), hermitian=op.hermitian)
    x = np.asarray(x, dtype=np.complex128)
    return (s @ x.ravel()).reshape(x.shape)


def error_estimate(op, x, k: int, ell: int, p: float | None = None) -> float:
    """eps = |x~ - x| / (2|x|) with x~ = sgn(sgn(x)) (Sec. 3)."""
    y, _ = sign_apply(op, x, k, ell, p)
    xt, _ = sign_apply(op, y, k, ell, p)
    return float(np.linalg.norm(xt - x) / (2 * np.linalg.norm(x)))


def rel_err(y, yref) -> float:
    return float(np.linalg.norm(np.ravel(y) - np.ravel(yref)) / np.linalg.norm(np.ravel(yref)))
