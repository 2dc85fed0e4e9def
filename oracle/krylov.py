"""Lanczos (App. A) and two-sided Lanczos (App. B) recurrences (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Both build the basis V_k of K_k(A, x) and the tridiagonal Ritz matrix H_k of
Sec. 3: H_k = V_k^dagger A V_k (orthonormal V_k, Hermitian A) or the two-sided
Ritz matrix H_k = W_k^dagger A V_k with biorthonormal W_k^dagger V_k = 1.

Readings where the paper is silent or ambiguous:

* k is rounded up to an even number (Sec. 4.2: odd sizes give spurious
  near-zero Ritz values); the loop stops after H(k,k), so exactly k basis
  vectors and k applications of A (and k of A^dagger when two-sided).
* Hermitian: H(j,j) = Re(v_j^dagger r) (the Ritz matrix is real symmetric,
  App. A, and steps 3-5 of App. C run in real arithmetic).
* Two-sided: beta = principal sqrt(delta), gamma = conj(delta)/beta.
* Breakdowns (thresholds unstated in App. A and B), with
  S_j = |H(j,j)| + |H(j,j-1) H(j-1,j)|^{1/2} and the basis norms
  ||v_{j+1}|| = ||r|| / |beta|, ||w_{j+1}|| = ||l|| / |gamma| carried along:
  - Hermitian lucky breakdown (invariant subspace): beta_j <= 1e-10 S_j
    -> stop with k_used = j, status "ok";
  - two-sided lucky breakdown: ||r|| <= 1e-8 S_j ||v_j|| or
    ||l|| <= 1e-8 S_j ||w_j|| -> stop with k_used = j, status "ok" (the
    looser threshold covers the rounding that the oblique basis amplifies);
  - serious: |delta| <= 1e-12 ||r|| ||l|| with r, l nonzero -> stop with
    k_used = j, status "breakdown" (App. B: serious breakdown, stop).
* No reorthogonalisation (App. A and B have none).
"""
from __future__ import annotations

import numpy as np

LUCKY_TAU_HERMITIAN = 1e-10
LUCKY_TAU_TWO_SIDED = 1e-8
SERIOUS_TAU = 1e-12


def even_up(k: int) -> int:
    k = int(k)
    return k + (k & 1)


class KrylovResult:
    def __init__(self, V, alpha, beta, gamma, k_used, status, bnorm, W=None):
        self.V = V              # n x k_used basis (columns v_j)
        self.W = W              # n x k_used left basis (two-sided) or None
        self.alpha = alpha      # diagonal H(j,j), length k_used
        self.beta = beta        # sub-diagonal H(j+1,j), length k_used-1
        self.gamma = gamma      # super-diagonal H(j,j+1), length k_used-1
        self.k_used = k_used
        self.status = status    # "ok", "breakdown", "zero"
        self.bnorm = bnorm      # |x|

    def H(self) -> np.ndarray:
        k = self.k_used
        h = np.zeros((k, k), dtype=np.result_type(self.alpha, self.beta, self.gamma))
        h[np.arange(k), np.arange(k)] = self.alpha
        if k > 1:
            h[np.arange(1, k), np.arange(k - 1)] = self.beta
            h[np.arange(k - 1), np.arange(1, k)] = self.gamma
        return h


def lanczos(matvec, x: np.ndarray, k: int, keep_basis: bool = True) -> KrylovResult:
    """App. A.  Returns V_k, the real diagonal alpha and off-diagonal beta.

    A real x (with a real symmetric operator) keeps the whole run in real
    arithmetic, as App. C asks for the inner level in the Hermitian case.
    """
    k = even_up(k)
    x = np.asarray(x)
    dtype = np.float64 if np.isrealobj(x) else np.complex128  # real for steps 3-5
    x = x.astype(dtype).ravel()
    n = x.size
    xn = float(np.linalg.norm(x))
    if xn == 0.0:
        return KrylovResult(np.zeros((n, 0), dtype), np.zeros(0), np.zeros(0),
                            np.zeros(0), 0, "zero", 0.0)
    V = np.zeros((n, k), dtype=dtype) if keep_basis else None
    alpha = np.zeros(k)
    beta = np.zeros(max(k - 1, 0))
    v = x / xn
    v_prev = None
    if keep_basis:
        V[:, 0] = v
    r = matvec(v)
    status, k_used = "ok", k
    for j in range(1, k + 1):           # j is the 1-based iteration index
        a = float(np.real(np.vdot(v, r)))
        alpha[j - 1] = a
        r = r - a * v
        if j == k:
            break
        b = float(np.linalg.norm(r))
        b_prev = beta[j - 2] if j >= 2 else 0.0
        if b <= LUCKY_TAU_HERMITIAN * (abs(a) + b_prev):
            k_used = j
            break
        beta[j - 1] = b
        v_prev, v = v, r / b
        if keep_basis:
            V[:, j] = v
        r = matvec(v) - b * v_prev
    alpha = alpha[:k_used]
    beta = beta[:max(k_used - 1, 0)]
    return KrylovResult(V[:, :k_used] if keep_basis else None, alpha, beta, beta.copy(),
                        k_used, status, xn)


def two_sided_lanczos(matvec, rmatvec, x: np.ndarray, k: int,
                      keep_basis: bool = True, keep_left: bool = False) -> KrylovResult:
    """App. B.  H(j+1,j) = beta_j, H(j,j+1) = gamma_j, W^dagger V = 1."""
    k = even_up(k)
    x = np.asarray(x, dtype=np.complex128).ravel()
    n = x.size
    xn = float(np.linalg.norm(x))
    if xn == 0.0:
        z = np.zeros(0, complex)
        return KrylovResult(np.zeros((n, 0), complex), z, z, z, 0, "zero", 0.0)
    V = np.zeros((n, k), dtype=np.complex128) if keep_basis else None
    W = np.zeros((n, k), dtype=np.complex128) if keep_left else None
    alpha = np.zeros(k, dtype=np.complex128)
    beta = np.zeros(max(k - 1, 0), dtype=np.complex128)
    gamma = np.zeros(max(k - 1, 0), dtype=np.complex128)
    v = x / xn
    w = v.copy()
    vnorm, wnorm = 1.0, 1.0
    if keep_basis:
        V[:, 0] = v
    if keep_left:
        W[:, 0] = w
    r = matvec(v)
    l = rmatvec(w)
    status, k_used = "ok", k
    for j in range(1, k + 1):
        a = np.vdot(w, r)
        alpha[j - 1] = a
        r = r - a * v
        l = l - np.conj(a) * w
        if j == k:
            break
        delta = np.vdot(r, l)
        nr = float(np.linalg.norm(r))
        nl = float(np.linalg.norm(l))
        s = abs(a) + (np.sqrt(abs(beta[j - 2] * gamma[j - 2])) if j >= 2 else 0.0)
        if nr <= LUCKY_TAU_TWO_SIDED * s * vnorm or nl <= LUCKY_TAU_TWO_SIDED * s * wnorm:
            k_used = j
            break
        if abs(delta) <= SERIOUS_TAU * nr * nl:
            k_used, status = j, "breakdown"
            break
        b = np.sqrt(delta)
        g = np.conj(delta) / b
        beta[j - 1] = b
        gamma[j - 1] = g
        v_prev, w_prev = v, w
        v = r / b
        w = l / np.conj(g)
        vnorm, wnorm = nr / abs(b), nl / abs(g)
        if keep_basis:
            V[:, j] = v
        if keep_left:
            W[:, j] = w
        r = matvec(v) - g * v_prev
        l = rmatvec(w) - np.conj(b) * w_prev
    alpha = alpha[:k_used]
    beta = beta[:max(k_used - 1, 0)]
    gamma = gamma[:max(k_used - 1, 0)]
    return KrylovResult(V[:, :k_used] if keep_basis else None, alpha, beta, gamma,
                        k_used, status, xn, W[:, :k_used] if keep_left else None)
