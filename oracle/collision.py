"""Collision probability of the p-stable (Gaussian) hash, Eq. (1) of Section 3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (1) gives, for two points at distance r and bucket width w,

    P(r) = integral_0^w (1/r) * (2/sqrt(2*pi)) * exp(-t^2 / (2 r^2)) * (1 - t/w) dt.

With s = w / r the integral has the closed form

    P(r) = 1 - 2*Phi(-s) - (2 / (sqrt(2*pi) * s)) * (1 - exp(-s^2 / 2)),

obtained by splitting (1 - t/w) and integrating the Gaussian density term by term
(the t-weighted term integrates exactly to r^2 (1 - exp(-s^2/2)) / w times the
normalisation).  Layer collision (k functions ANDed) is P^k; the chance to meet
in at least one of L layers (ORed) is 1 - (1 - P^k)^L, by the independence of the
functions (Section 1.1).
"""
from __future__ import annotations

import math


def _phi_neg(s: float) -> float:
    """Phi(-s) for the standard normal CDF Phi."""
    return 0.5 * math.erfc(s / math.sqrt(2.0))


def p_collide(r: float, w: float) -> float:
    """Single-function collision probability P(r) of Eq. (1) (closed form)."""
    if r <= 0:
        return 1.0
    s = w / r
    return 1.0 - 2.0 * _phi_neg(s) - (2.0 / (math.sqrt(2.0 * math.pi) * s)) * (1.0 - math.exp(-s * s / 2.0))


def p_layer(r: float, w: float, k: int) -> float:
    """Probability that all k functions of one layer collide."""
    return p_collide(r, w) ** k


def p_candidate(r: float, w: float, k: int, L: int) -> float:
    """Probability that a point at distance r is a candidate in at least one of L layers."""
    return 1.0 - (1.0 - p_layer(r, w, k)) ** L
