"""The overlap operator built on the sign function (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2, Eq. Dovmu: D_ov(mu) = 1 + gamma5 sgn(gamma5 D_w(mu)), with A =
gamma5 D_w(mu) the operator of ``dirac.Operator`` and gamma5 acting on the
spin index of every site (``dirac.gamma5_full``).
"""
from __future__ import annotations

import numpy as np

from . import dirac, nested
from .signfun import sign_eig


def from_sign(op, x, sx):
    """x + gamma5 (sgn(A) x), given sx = sgn(A) x."""
    V = op.n // 12
    g5 = dirac.gamma5_full(V)
    x = np.asarray(x, dtype=np.complex128).ravel()
    return x + g5 @ np.asarray(sx, dtype=np.complex128).ravel()


def overlap_apply(op, x, k: int, ell: int, p: float | None = None):
    """D_ov x with sgn(A) x from the nested Krylov-Ritz method (Eq. nested)."""
    y, _ = nested.sign_apply(op, x, k, ell, p=p)
    return from_sign(op, x, y)


def overlap_dense(op):
    """The dense D_ov(mu) from the spectral sign of A (Eq. fAdef)."""
    V = op.n // 12
    g5 = dirac.gamma5_full(V).toarray()
    return np.eye(op.n) + g5 @ sign_eig(op.dense(), hermitian=op.hermitian)
