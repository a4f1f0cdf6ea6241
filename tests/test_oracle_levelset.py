"""Pins of the level-set example (Dziuk's surface) on the CPU.

* The closed-form right-hand side in workloads (curvature form of -Lap_S u) equals the
  paper's recipe f = -div_S(grad_S u) + u, with div_S v = div v - sum_j (grad v_j . n) n_j,
  derived symbolically with SymPy, at random surface points.
* Points p + t n(p) within the reach map back to p exactly (closed form).
* Beyond the reach (h = 1/16) the band's surface points lie on S and are stationary, are at
  most slightly farther than a dense random sampling, and the exclusion filter drops no node
  that the sampling puts in the band.
* The V-cycle on the level set converges and its limit is second-order accurate.
"""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import geometry as og
from oracle import vcycle as ov


def _surface_points(m, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((m, 3))
    V /= np.linalg.norm(V, axis=1)[:, None]
    return np.stack([V[:, 0] + V[:, 2] ** 2, V[:, 1], V[:, 2]], axis=1)


def _phi(Y):
    p = Y[:, 0] - Y[:, 2] ** 2
    return p * p + Y[:, 1] ** 2 + Y[:, 2] ** 2 - 1.0


def test_rhs_matches_symbolic_surface_divergence():
    sp = pytest.importorskip("sympy")
    x1, x2, x3 = sp.symbols("x1 x2 x3", real=True)
    X = sp.Matrix([x1, x2, x3])
    phi = (x1 - x3 ** 2) ** 2 + x2 ** 2 + x3 ** 2 - 1
    g = sp.Matrix([sp.diff(phi, v) for v in X])
    n = g / sp.sqrt(g.dot(g))
    u = x1 * x2
    gu = sp.Matrix([sp.diff(u, v) for v in X])
    v = gu - gu.dot(n) * n
    div = sum(sp.diff(v[j], X[j]) for j in range(3))
    corr = sum(sp.Matrix([sp.diff(v[j], X[k]) for k in range(3)]).dot(n) * n[j] for j in range(3))
    f_sym = sp.lambdify((x1, x2, x3), -(div - corr) + u, "numpy")
    Y = _surface_points(200, 11)
    assert np.max(np.abs(_phi(Y))) < 1e-12
    f = W.dziuk_x1x2().f(Y)
    ref = f_sym(Y[:, 0], Y[:, 1], Y[:, 2])
    assert np.max(np.abs(f - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_samples_on_surface():
    S = og.dziuk_samples()
    assert S.shape == (6 * og.DZIUK_SAMPLES_K ** 2, 3)
    assert np.max(np.abs(_phi(S))) < 1e-14


def test_newton_closest_point_exact_within_reach():
    """x = p + t n(p) with |t| below the reach has closest point p and distance |t|."""
    P = _surface_points(20000, 3)
    p = P[:, 0] - P[:, 2] ** 2
    g = np.stack([2 * p, 2 * P[:, 1], 2 * P[:, 2] - 4 * P[:, 2] * p], axis=1)
    n = g / np.linalg.norm(g, axis=1)[:, None]
    t = np.random.default_rng(4).uniform(-0.05, 0.05, P.shape[0])
    X = P + t[:, None] * n
    cp, d2, unconv = og._dziuk_newton(X, 0.06 ** 2)
    assert not np.any(unconv)
    assert np.max(np.abs(cp - P)) < 1e-12
    assert np.max(np.abs(np.sqrt(d2) - np.abs(t))) < 1e-12


def test_band_h16_against_sampling():
    """Beyond the reach (h = 1/16) the band still contains every node within the band radius
    of a dense surface sampling, its surface points are on S, and they are at most a little
    farther than the sampled distance."""
    from scipy.spatial import cKDTree

    h = 1.0 / 16
    lev = ob.build_level(W.dziuk_surface(), h, W.LAM2_3D)
    X = lev.idx * h
    cp = lev.cp
    assert np.max(np.abs(_phi(cp))) < 1e-12
    p = cp[:, 0] - cp[:, 2] ** 2
    g = np.stack([2 * p, 2 * cp[:, 1], 2 * cp[:, 2] - 4 * cp[:, 2] * p], axis=1)
    cr = np.linalg.norm(np.cross(X - cp, g), axis=1) / np.linalg.norm(g, axis=1)
    assert np.mean(cr < 1e-11) > 0.999  # stationary points (the rest keep a surface sample)
    T = cKDTree(_surface_points(600_000, 7))
    bf, _ = T.query(X)
    assert np.max(np.linalg.norm(X - cp, axis=1) - bf) < 2e-3
    box = np.stack(np.meshgrid(*[np.arange(lev.lo[a], lev.lo[a] + lev.ext[a]) for a in range(3)], indexing="ij"),
                   axis=-1).reshape(-1, 3)
    bfb, _ = T.query(box * h)
    inside = bfb ** 2 <= W.LAM2_3D * h * h * 0.99
    assert np.all(lev.lookup(box[inside]) >= 0)


def test_levelset_solve_second_order():
    prob = W.dziuk_x1x2()
    errs = []
    for hinv, levels in ((16, 2), (32, 3)):
        H = ob.build_hierarchy(prob.surface, 1.0 / hinv, levels, W.LAM2_3D)
        cp = H.levels[0].cp
        res = ov.solve(H, prob.f(cp), ov.Params(), rtol=1e-10, max_cycles=60)
        assert res.relres[-1] < 1e-10
        assert ov.contraction(res.relres) < 0.4
        errs.append(np.max(np.abs(res.u - prob.u_exact(cp))))
    assert 3.0 < errs[0] / errs[1] < 5.5, errs
