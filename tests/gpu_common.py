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
