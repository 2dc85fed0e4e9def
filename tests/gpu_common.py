"""Helpers shared by the GPU parity tests (inputs come from nks_inputs,
expected values from the oracle; nothing here computes the method)."""
import functools

import numpy as np

import nks_inputs as I

M0 = 1.6


def rel(a, b) -> float:
    a = np.ravel(np.asarray(a))
    b = np.ravel(np.asarray(b))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@functools.lru_cache(maxsize=None)
def ctx():
    import paper_0912_4457_amd as nks
    return nks.Context(0)


@functools.lru_cache(maxsize=None)
def links(dims, eps, seed):
    return I.su3_links(dims, eps, seed)


@functools.lru_cache(maxsize=None)
def lattice(dims, eps, seed, mu, kind="su3"):
    import paper_0912_4457_amd as nks
    if kind == "su3":
        u = links(dims, eps, seed)
    elif kind == "unit":
        u = I.unit_links(dims)
    elif kind == "pure":
        u = I.pure_gauge_links(I.random_su3_field(dims, seed))
    else:
        raise ValueError(kind)
    return nks.Lattice(ctx(), dims, u, m0=M0, mu=mu)


@functools.lru_cache(maxsize=None)
def operator(dims, eps, seed, mu, kind="su3"):
    from oracle import dirac
    if kind == "su3":
        u = links(dims, eps, seed)
    elif kind == "unit":
        u = I.unit_links(dims)
    else:
        u = I.pure_gauge_links(I.random_su3_field(dims, seed))
    return dirac.Operator(u, dims, M0, mu)


def to_np(t):
    return t.detach().cpu().numpy()


def rounding_tolerance(run, b, hermitian, floor=1e-10, factor=10.0, draws=3):
    """(tolerance, response) for a GPU result that equals the oracle's run(b)
    up to rounding.  Hermitian runs take ``floor``.  Two-sided runs (Eq.
    non-nested-oblique, App. B) amplify rounding well beyond that, so any
    other rounding order lands further than 1e-10 away: their tolerance is
    ``factor`` times the oracle's own response to two-ulp changes of every
    component of the source (relative to the entry, plus the same relative to
    the source's rms entry, so that a point source is not merely rescaled),
    at least ``floor``."""
    if hermitian:
        return floor, 0.0
    b = np.asarray(b, dtype=np.complex128)
    y0 = np.ravel(run(b))
    resp = 0.0
    for s in range(draws):
        rng = np.random.default_rng(7100 + s)
        rms = float(np.linalg.norm(b)) / np.sqrt(b.size)
        bp = b * (1 + 4e-16 * rng.choice([-1.0, 1.0], b.shape)) + 4e-16 * rms * rng.choice([-1.0, 1.0], b.shape)
        resp = max(resp, rel(run(bp), y0))
    return max(floor, factor * resp), resp
