"""Closest-point functions (Sec. 2.1: cp maps a point of the tubular neighbourhood to a
nearest surface point) for the analytic surfaces used in the paper's examples.

Floating-point convention (shared *as a convention* with the GPU library's band builder,
so that band membership and stencil bases agree bit for bit): plain IEEE double
operations in exactly the order written below, no fused multiply-add, correctly rounded
sqrt and division.  Ties (points where cp is not unique) are broken so that the chosen
point lies on the surface:

* circle / sphere centre: direction (1, 0, 0)
* torus axis (rho = 0): radial direction (1, 0, 0)
* torus tube-centre circle: tube direction = outward radial direction
"""
from __future__ import annotations

import numpy as np

from workloads import CIRCLE, SPHERE, TORUS, Surface


def closest_point_and_dist2(s: Surface, X: np.ndarray):
    """Return (cp, dist^2) for points X (m x d)."""
    X = np.asarray(X, dtype=np.float64)
    c = s.c0()
    if s.kind in (CIRCLE, SPHERE):
        D = X - c
        if s.dim == 2:
            rho2 = D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]
        else:
            rho2 = (D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2]
        rho = np.sqrt(rho2)
        zero = rho == 0.0
        safe = np.where(zero, 1.0, rho)
        N = D / safe[:, None]
        N[zero] = 0.0
        N[zero, 0] = 1.0
        cp = c + s.R * N
        d = rho - s.R
        return cp, d * d
    if s.kind == TORUS:
        D = X - c
        rho = np.sqrt(D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1])
        zero = rho == 0.0
        safe = np.where(zero, 1.0, rho)
        ex = np.where(zero, 1.0, D[:, 0] / safe)
        ey = np.where(zero, 0.0, D[:, 1] / safe)
        a = rho - s.R
        b = D[:, 2]
        t = np.sqrt(a * a + b * b)
        tz = t == 0.0
        tsafe = np.where(tz, 1.0, t)
        na = np.where(tz, 1.0, a / tsafe)
        nb = np.where(tz, 0.0, b / tsafe)
        rad = s.R + s.r * na
        cp = np.stack([c[0] + rad * ex, c[1] + rad * ey, c[2] + s.r * nb], axis=1)
        d = t - s.r
        return cp, d * d
    raise ValueError("unknown surface kind %r" % s.kind)


def closest_point(s: Surface, X: np.ndarray) -> np.ndarray:
    return closest_point_and_dist2(s, X)[0]


def bounding_box(s: Surface):
    """Axis-aligned box containing the surface."""
    c = s.c0()
    if s.kind in (CIRCLE, SPHERE):
        ext = np.full(s.dim, s.R)
    else:
        ext = np.array([s.R + s.r, s.R + s.r, s.r])
    return c - ext, c + ext
