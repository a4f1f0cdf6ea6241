"""Closest-point functions (Sec. 2.1: cp maps a point of the tubular neighbourhood to a
nearest surface point) for the analytic surfaces used in the paper's examples, and the
Newton closest point of the level-set example (Dziuk's surface, Sec. 4.6.5).

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

from workloads import CIRCLE, DZIUK, SPHERE, TORUS, Surface

#: Newton iterations of the level-set closest point (quadratic convergence reaches the
#: double-precision floor in 5-7 steps; the rest change nothing beyond the last bit)
NEWTON_ITERS = 25
#: the Newton start is the nearest of 6 K^2 surface samples: cube-face grid points
#: (1, u, v), ... with u, v = (2 i + 1) / K - 1, normalised onto the unit sphere and bent
#: onto Dziuk's surface by y1 = v1 + v3^2 (only +, *, / and sqrt, so exactly reproducible)
DZIUK_SAMPLES_K = 16


def dziuk_samples(K: int = DZIUK_SAMPLES_K) -> np.ndarray:
    t = (2.0 * np.arange(K) + 1.0) / K - 1.0
    U, V = np.meshgrid(t, t, indexing="ij")
    U, V = U.ravel(), V.ravel()
    O = np.ones_like(U)
    P = np.concatenate([np.stack(f, axis=1) for f in
                        ((O, U, V), (-O, U, V), (U, O, V), (U, -O, V), (U, V, O), (U, V, -O))])
    r = np.sqrt((P[:, 0] * P[:, 0] + P[:, 1] * P[:, 1]) + P[:, 2] * P[:, 2])
    Q = P / r[:, None]
    return np.stack([Q[:, 0] + Q[:, 2] * Q[:, 2], Q[:, 1], Q[:, 2]], axis=1)


def _dziuk_newton(X: np.ndarray, thr: float):
    """Closest points on the level set phi(y) = (y1 - y3^2)^2 + y2^2 + y3^2 - 1 = 0 by Newton's
    method on the stationarity conditions of |y - x|^2 under phi(y) = 0 (the paper's level-set
    example minimises the squared distance with Newton's method):

        F(y, mu) = (y - x + mu grad(phi)(y), phi(y)) = 0,
        J = [[K, g], [g^T, 0]],  K = I + mu Hess(phi)(y),  g = grad(phi)(y),

    started from the nearest surface sample (lowest index on ties), with the multiplier
    mu = (x - y) . g / |g|^2 of that sample.  A global start is needed: the coarse bands reach
    beyond the surface's reach, where a local start (the projection of x) can converge to a
    stationary point that is not the closest point and leave holes in the band.  K couples y1
    and y3 only, so each step is solved in closed form: dmu = (F_phi - g^T K^-1 F_y) /
    (g^T K^-1 g), dy = -K^-1 (F_y + g dmu).  Points that provably have no surface point within
    sqrt(thr) (a Lipschitz bound, below) are not iterated (dist2 = inf).  A point whose
    iteration does not converge, or converges to a stationary point farther than its start
    (beyond the reach, between two nearly equidistant sheets), keeps its start, the nearest
    sample, as its surface point, so the band has no holes.  Convergence means |phi| <= 1e-12
    and every stationarity residual <= 1e-12.  Returns (cp, dist2, unconverged)."""
    x1, x2, x3 = X[:, 0], X[:, 1], X[:, 2]
    p0 = x1 - x3 * x3
    ph = (p0 * p0 + x2 * x2) + (x3 * x3 - 1.0)
    # rigorous exclusion: on the ball |y - x| <= r (r^2 = thr) the gradient is bounded by G
    # (|y3| <= |x3| + r, |y2| <= |x2| + r, |y1 - y3^2| <= |p| + r + 2 |x3| r + r^2 =: P,
    # |g|^2 <= 4 P^2 + 4 Y2^2 + Y3^2 (2 + 4 P)^2), so |phi(x)| > G r means no surface point
    # within r; every other point is solved
    r = np.sqrt(thr) if np.isfinite(thr) else np.inf
    ax3 = np.abs(x3)
    P = ((np.abs(p0) + r) + (2.0 * ax3) * r) + r * r
    Y2 = np.abs(x2) + r
    Y3 = ax3 + r
    q = 2.0 + 4.0 * P
    G2 = (4.0 * (P * P) + 4.0 * (Y2 * Y2)) + (Y3 * Y3) * (q * q)
    near = ph * ph <= G2 * thr
    Z = X[near]
    S = dziuk_samples()
    best = np.empty(Z.shape[0], dtype=np.int64)
    for c0 in range(0, Z.shape[0], 2048):
        z = Z[c0:c0 + 2048]
        d0 = S[None, :, 0] - z[:, None, 0]
        d1 = S[None, :, 1] - z[:, None, 1]
        d2 = S[None, :, 2] - z[:, None, 2]
        best[c0:c0 + 2048] = np.argmin((d0 * d0 + d1 * d1) + d2 * d2, axis=1)
    z1, z2, z3 = Z[:, 0], Z[:, 1], Z[:, 2]
    y1, y2, y3 = S[best, 0].copy(), S[best, 1].copy(), S[best, 2].copy()
    with np.errstate(all="ignore"):
        p = y1 - y3 * y3
        g1 = 2.0 * p
        g2 = 2.0 * y2
        g3 = 2.0 * y3 - 4.0 * y3 * p
        gg = (g1 * g1 + g2 * g2) + g3 * g3
        mu = (((z1 - y1) * g1 + (z2 - y2) * g2) + (z3 - y3) * g3) / gg
        for _ in range(NEWTON_ITERS):
            p = y1 - y3 * y3
            g1 = 2.0 * p
            g2 = 2.0 * y2
            g3 = 2.0 * y3 - 4.0 * y3 * p
            ph = (p * p + y2 * y2) + (y3 * y3 - 1.0)
            F1 = (y1 - z1) + mu * g1
            F2 = (y2 - z2) + mu * g2
            F3 = (y3 - z3) + mu * g3
            h33 = (2.0 - 4.0 * p) + 8.0 * (y3 * y3)
            a = 1.0 + 2.0 * mu
            b = (-4.0 * mu) * y3
            d = 1.0 + mu * h33
            det = a * d - b * b
            kf1 = (d * F1 - b * F3) / det
            kf3 = (a * F3 - b * F1) / det
            kf2 = F2 / a
            kg1 = (d * g1 - b * g3) / det
            kg3 = (a * g3 - b * g1) / det
            kg2 = g2 / a
            gkf = (g1 * kf1 + g2 * kf2) + g3 * kf3
            gkg = (g1 * kg1 + g2 * kg2) + g3 * kg3
            dmu = (ph - gkf) / gkg
            y1 = y1 - (kf1 + kg1 * dmu)
            y2 = y2 - (kf2 + kg2 * dmu)
            y3 = y3 - (kf3 + kg3 * dmu)
            mu = mu + dmu
        p = y1 - y3 * y3
        ph = (p * p + y2 * y2) + (y3 * y3 - 1.0)
        r1 = (y1 - z1) + mu * (2.0 * p)
        r2 = (y2 - z2) + mu * (2.0 * y2)
        r3 = (y3 - z3) + mu * (2.0 * y3 - 4.0 * y3 * p)
        e1, e2, e3 = y1 - z1, y2 - z2, y3 - z3
        dn = (e1 * e1 + e2 * e2) + e3 * e3
    conv = (np.abs(ph) <= 1e-12) & (np.maximum(np.maximum(np.abs(r1), np.abs(r2)), np.abs(r3)) <= 1e-12)
    # unconverged, or converged to a stationary point farther than the start: keep the start
    # (a surface sample) as the node's surface point
    s1, s2, s3 = S[best, 0], S[best, 1], S[best, 2]
    f1, f2, f3 = s1 - z1, s2 - z2, s3 - z3
    ds = (f1 * f1 + f2 * f2) + f3 * f3
    use = conv & (dn <= ds)
    cp = X.copy()
    dist2 = np.full(X.shape[0], np.inf)
    unconv = np.zeros(X.shape[0], dtype=bool)
    cp[near, 0] = np.where(use, y1, s1)
    cp[near, 1] = np.where(use, y2, s2)
    cp[near, 2] = np.where(use, y3, s3)
    dist2[near] = np.where(use, dn, ds)
    unconv[near] = ~conv
    return cp, dist2, unconv


def closest_point_and_dist2(s: Surface, X: np.ndarray, thr: float = np.inf):
    """Return (cp, dist^2) for points X (m x d).  thr (the squared band radius) only matters
    for level sets: points far beyond it get dist^2 = inf without a Newton solve, and a point
    within it whose Newton iteration fails raises."""
    X = np.asarray(X, dtype=np.float64)
    c = s.c0()
    if s.kind == DZIUK:
        cp, dist2, _ = _dziuk_newton(X - c, thr)
        return cp + c, dist2
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
    elif s.kind == DZIUK:
        # x1 = x3^2 +- sqrt(1 - x2^2 - x3^2) lies in [-1, 5/4]; |x2|, |x3| <= 1
        return c + np.array([-1.0, -1.0, -1.0]), c + np.array([1.25, 1.0, 1.0])
    else:
        ext = np.array([s.R + s.r, s.R + s.r, s.r])
    return c - ext, c + ext
