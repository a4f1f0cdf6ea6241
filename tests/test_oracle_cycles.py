"""Pins of the W-cycle and the full-multigrid start in the oracle (CPU).

* The W-cycle (cycle index 2) has the V-cycle's fixed point (the sparse direct solution) and
  contracts at least as fast per cycle.
* The full-multigrid start (nested iteration from the coarsest level) is already within a
  small factor of the discretization error (the classical FMG property), and the solve from
  it reaches the same fixed point in fewer cycles than from u = 0; so does the mixed-precision
  refinement started from it.
"""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import direct as od
from oracle import vcycle as ov


def _hier(cfg):
    return ob.build_hierarchy(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)


@pytest.mark.parametrize("cfg", [W.config_circle(64, 4), W.config_sphere(16, 3)], ids=["circle64", "sphere16"])
def test_w_cycle_fixed_point_and_rate(cfg):
    H = _hier(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    v = ov.solve(H, f, ov.Params(), rtol=1e-12, max_cycles=80)
    w = ov.solve(H, f, ov.Params(gamma=2), rtol=1e-12, max_cycles=80)
    u_star = od.solve_direct(H.levels[0], H.E[0] @ f, 1.0)
    assert np.max(np.abs(w.u - u_star)) <= 1e-10 * np.max(np.abs(u_star))
    assert ov.contraction(w.relres) <= ov.contraction(v.relres) + 1e-3
    assert w.cycles <= v.cycles


@pytest.mark.parametrize("cfg", [W.config_circle(64, 4), W.config_sphere(32, 4)], ids=["circle64", "sphere32"])
def test_fmg_start_reaches_discretization_error(cfg):
    H = _hier(cfg)
    cp = H.levels[0].cp
    f = cfg.problem.f(cp)
    p = ov.Params()
    coarse = ov.CoarseSolver(H, p)
    u_fmg = ov.fmg_start(H, f, p, coarse)
    conv = ov.solve(H, f, p, rtol=1e-11, max_cycles=80)
    e_fmg = np.max(np.abs(u_fmg - cfg.problem.u_exact(cp)))
    e_conv = np.max(np.abs(conv.u - cfg.problem.u_exact(cp)))
    assert e_fmg < 3.0 * e_conv, (e_fmg, e_conv)
    from_fmg = ov.solve(H, f, p, rtol=1e-11, max_cycles=80, fmg=True)
    assert from_fmg.cycles < conv.cycles
    assert np.max(np.abs(from_fmg.u - conv.u)) <= 1e-9 * np.max(np.abs(conv.u))


def test_mixed_solve_from_fmg_start_reaches_the_direct_solution():
    """The mixed-precision refinement started from the float64 full-multigrid start reaches
    the sparse direct solution of A u = E f (its float64 residual decides the fixed point)
    in fewer outer cycles than from u = 0."""
    from oracle import mixed as omx

    cfg = W.config_circle(64, 4)
    H = _hier(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    p = ov.Params()
    u0 = ov.fmg_start(H, f, p, ov.CoarseSolver(H, p))
    from0 = omx.solve_mixed(H, f, p, rtol=1e-10, max_cycles=60)
    fromf = omx.solve_mixed(H, f, p, rtol=1e-10, max_cycles=60, u0=u0)
    u_star = od.solve_direct(H.levels[0], H.E[0] @ f, 1.0)
    assert fromf.relres[-1] < 1e-10
    assert np.max(np.abs(fromf.u - u_star)) <= 1e-9 * np.max(np.abs(u_star))
    assert len(fromf.relres) < len(from0.relres)
