"""Pins of the oracle's multi-level nesting (Sec. 4.5, Fig. 12): the one-level
case is the nested method, full-size levels give the exact sign of H_k, p
tends to 1 with depth, the error converges in the innermost size to the
one-level error, and the result meets the pure-gauge closed form."""
import numpy as np
import pytest

import nks_inputs as I
from oracle import closedform, dirac, krylov, multilevel, nested, signfun

M0 = 1.6
_CACHE = {}


def _setup(mu, k=300):
    key = (mu, k)
    if key not in _CACHE:
        dims = (3, 3, 3, 3)
        op = dirac.Operator(I.su3_links(dims, 0.2, 31), dims, M0, mu)
        b = I.gaussian_source(dims, 3).ravel()
        ref = signfun.sign_eig(op.dense(), hermitian=op.hermitian) @ b
        if op.hermitian:
            kr = krylov.lanczos(op.matvec, b, k)
        else:
            kr = krylov.two_sided_lanczos(op.matvec, op.rmatvec, b, k)
        _CACHE[key] = (op, kr, ref)
    return _CACHE[key]


def _err(kr, c, ref):
    return nested.rel_err(kr.bnorm * (kr.V @ c), ref)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_one_level_is_the_nested_method(mu):
    op, kr, _ = _setup(mu)
    c1, i1 = nested.nested_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, 60)
    cm, im = multilevel.multilevel_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, [60])
    assert im["sizes"] == [300, 60] and im["p"] == [i1["p"]]
    assert np.array_equal(c1, cm)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_full_size_levels_give_the_sign_of_H(mu):
    # a level whose inner space is the whole space is exact (Eq. innersign with
    # W_i square, and sgn(T') = sgn(T) by Eq. proofprec), at any depth
    op, kr, _ = _setup(mu)
    k = 24
    a, b, g = kr.alpha[:k], kr.beta[:k - 1], kr.gamma[:k - 1]
    H = np.diag(a) + np.diag(b, -1) + np.diag(g, 1)
    s = signfun.sign_eig(H, hermitian=op.hermitian)[:, 0]
    for levels in (1, 2, 3):
        c, info = multilevel.multilevel_coefficients(a, b, g, op.hermitian, [k] * levels, force_nested=True)
        assert info["sizes"] == [k] * (levels + 1)
        assert np.linalg.norm(c - s) <= 1e-12 * np.linalg.norm(s)
    # without force_nested the first full-size level stops the recursion: RHi on H
    c, info = multilevel.multilevel_coefficients(a, b, g, op.hermitian, [k, 8])
    assert info["levels"] == 0 and np.linalg.norm(c - s) <= 1e-12 * np.linalg.norm(s)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_p_tends_to_one_with_depth(mu):
    # footnote of Sec. 4.5: the p factor converges to 1 as levels are added
    op, kr, _ = _setup(mu)
    _, info = multilevel.multilevel_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, [60, 20, 8, 4, 2])
    dev = np.abs(np.log(info["p"]))
    assert np.all(np.diff(dev) < 0), info["p"]
    assert dev[-1] < 1e-3
    # each p is Eq. popt on the Ritz extremes of its own level
    for p, zmin, zmax in zip(info["p"], info["z_min"], info["z_max"]):
        assert p == pytest.approx(1.0 / np.sqrt(zmin * zmax), rel=1e-14)


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_innermost_size_convergence(mu):
    # Fig. 12: with the outer levels fixed in their convergence region the
    # error falls with the innermost size to the one-level error; five levels
    # with sizes 60 -> 20 -> 8 -> 4 -> 2 reach it (the sign of a 2 x 2 matrix)
    op, kr, ref = _setup(mu)
    c1, _ = nested.nested_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, 60)
    e1 = _err(kr, c1, ref)
    errs = []
    for k2 in (4, 8, 16):
        c, _ = multilevel.multilevel_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, [60, k2])
        errs.append(_err(kr, c, ref))
    assert errs[0] > 100 * errs[1] and errs[1] > 10 * errs[2]
    assert errs[2] <= 1.5 * e1 + 1e-13
    c5, info = multilevel.multilevel_coefficients(kr.alpha, kr.beta, kr.gamma, op.hermitian, [60, 20, 8, 4, 2])
    assert info["sizes"] == [300, 60, 20, 8, 4, 2] and info["levels"] == 5
    assert _err(kr, c5, ref) <= 1.5 * e1 + 1e-13


def test_multilevel_meets_pure_gauge_closed_form():
    dims = (4, 4, 4, 4)
    g = I.random_su3_field(dims, 44)
    for mu in (0.0, 0.3):
        op = dirac.Operator(I.pure_gauge_links(g), dims, M0, mu)
        b = I.gaussian_source(dims, 45)
        ref = closedform.pure_gauge_sign_apply(b, g, dims, M0, mu)
        y, info = multilevel.sign_apply(op, b, 200, [80, 20, 8])
        assert info["levels"] == 3
        assert nested.rel_err(y, ref) < 1e-10
