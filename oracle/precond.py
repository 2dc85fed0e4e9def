"""Preconditioning formulas of Sec. 4.1 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Eq. precond: z -> z' = (p z + 1/(p z)) / 2, sign-preserving (Eq. proofprec).
* Eq. popt: p_opt = (z_min z_max)^{-1/2} with z = |eigenvalue|.
* Hermitian: z'_max and the condition-number gain F of Eq. condimp.
* Circles C(+-m, r): p_opt = (m^2 - r^2)^{-1/2}, m' and r' of the mapped
  circle, relative distances d and d', and F of Eq. condimpNH.
* Ellipses E(+-m, a, b): p_opt = (m^2 - a^2)^{-1/2}.
"""
from __future__ import annotations

import numpy as np


def precond_map(z, p: float):
    z = np.asarray(z, dtype=np.complex128)
    return 0.5 * (p * z + 1.0 / (p * z))


def p_opt(z_min: float, z_max: float) -> float:
    return 1.0 / np.sqrt(z_min * z_max)


def zprime_max(z_min: float, z_max: float) -> float:
    r = np.sqrt(z_max / z_min)
    return 0.5 * (r + 1.0 / r)


def gain_hermitian(z_min: float, z_max: float) -> float:
    """F = C / C' of Eq. condimp (exact form, before the approximation)."""
    return (z_max / z_min) / zprime_max(z_min, z_max)


def gain_hermitian_approx(z_min: float, z_max: float) -> float:
    return 2.0 * np.sqrt(z_max / z_min)


def circle_p_opt(m: float, r: float) -> float:
    return 1.0 / np.sqrt(m * m - r * r)


def circle_image(m: float, r: float):
    """(m', r') of the image of C(m, r) under the map with p = p_opt."""
    ms = circle_p_opt(m, r) * m
    return 0.5 * (ms + 1.0 / ms), 0.5 * (ms - 1.0 / ms)


def circle_distances(m: float, r: float):
    """(d, d') = relative distances to the imaginary axis before and after."""
    d = (m - r) / (m + r)
    mp, rp = circle_image(m, r)
    dp = (mp - rp) / (mp + rp)
    return d, dp


def gain_circle(m: float, r: float) -> float:
    """F = d'/d of Eq. condimpNH, written as ((m + r)/m)^2."""
    return ((m + r) / m) ** 2


def gain_circle_gap(m: float, gap: float) -> float:
    """F = (2 - Delta/m)^2 with r = m - Delta."""
    return (2.0 - gap / m) ** 2


def ellipse_p_opt(m: float, a: float) -> float:
    return 1.0 / np.sqrt(m * m - a * a)
