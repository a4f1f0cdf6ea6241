"""Pins of the oracle's variable-coefficient operator and V-cycle on the CPU.

* a = 1 reduces every step to the constant-coefficient oracle (iterates equal).
* The flux form L~ is exact for a linear coefficient and a quadratic u at every node whose
  axis neighbours are in the band (closed form div(a grad u) = grad a . grad u + a Lap u).
* The V-cycle's fixed point is the sparse direct solution of the fine level's fixed-point
  equation (I - E D^{-1} N~) u = E D^{-1} f.
* On the paper's sphere example (a = cos(phi) + 1.5, u = cos(phi)) the limit is second-order
  accurate and the cycle contracts like the Poisson cycle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import varcoef as vc
from oracle import vcycle as ov


def _hier(cfg):
    return ob.build_hierarchy(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)


@pytest.mark.parametrize("cfg", [W.config_circle(32, 3), W.config_sphere(16, 2)], ids=["circle32", "sphere16"])
def test_unit_coefficient_is_the_poisson_cycle(cfg):
    H = _hier(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ones = [np.ones(lev.n) for lev in H.levels]
    a = vc.solve(H, ones, f, vc.VCParams(), rtol=0.0, max_cycles=4, keep_iterates=True)
    b = ov.solve(H, f, ov.Params(), rtol=0.0, max_cycles=4, keep_iterates=True)
    for k in range(4):
        # equal up to rounding (the coarsest LU factors differ by the scaling delta)
        assert np.max(np.abs(a.iterates[k] - b.iterates[k])) <= 1e-12 * np.max(np.abs(b.iterates[k]))
        assert abs(a.relres[k] - b.relres[k]) <= 1e-9 * b.relres[k]


def test_flux_form_exact_for_linear_coefficient():
    cfg = W.config_sphere(16, 2)
    H = _hier(cfg)
    lev = H.levels[0]
    X = lev.idx * lev.h
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    u = x * x + 2.0 * y * y - z * z + 0.5 * x * y
    a = 1.0 + 0.3 * x - 0.2 * y + 0.1 * z
    exact = 0.3 * (2 * x + 0.5 * y) - 0.2 * (4 * y + 0.5 * x) + 0.1 * (-2 * z) + a * (2.0 + 4.0 - 2.0)
    Nt, sigma = vc.flux_operator(lev, a)
    Lu = Nt @ u - sigma * u
    full = np.all(ob.neighbour_indices(lev) >= 0, axis=1)
    assert full.sum() > lev.n // 2
    assert np.max(np.abs(Lu[full] - exact[full])) <= 1e-9 * np.max(np.abs(exact))


@pytest.mark.parametrize("cfg", [W.config_circle(64, 3), W.config_sphere(12, 2)], ids=["circle64", "sphere12"])
def test_fixed_point_is_direct_solve(cfg):
    H = _hier(cfg)
    if H.levels[0].dim == 2:
        a_lv = [1.2 + 0.5 * lev.cp[:, 0] - 0.3 * lev.cp[:, 1] for lev in H.levels]
        f = cfg.problem.f(H.levels[0].cp)
    else:
        prob = W.sphere_varcoef()
        a_lv = [prob.a(lev.cp) for lev in H.levels]
        f = prob.f(H.levels[0].cp)
    res = vc.solve(H, a_lv, f, vc.VCParams(), rtol=1e-13, max_cycles=80)
    u_star = vc.fixed_point(H, a_lv, f, vc.VCParams())
    assert np.max(np.abs(res.u - u_star)) <= 1e-11 * np.max(np.abs(u_star))


def test_paper_sphere_example_second_order():
    prob = W.sphere_varcoef()
    errs, rates = [], []
    for hinv, levels in ((16, 3), (32, 4)):
        H = ob.build_hierarchy(prob.surface, 1.0 / hinv, levels, W.LAM2_3D)
        cp = H.levels[0].cp
        a_lv = [prob.a(lev.cp) for lev in H.levels]
        res = vc.solve(H, a_lv, prob.f(cp), vc.VCParams(), rtol=1e-10, max_cycles=60)
        assert res.relres[-1] < 1e-10
        rates.append(ov.contraction(res.relres))
        errs.append(np.max(np.abs(res.u - prob.u_exact(cp))))
    assert 3.0 < errs[0] / errs[1] < 5.5, errs
    assert max(rates) < 0.6, rates
