"""Pins of the oracle's standard-relaxation V-cycle (Sec. 4.5) on the CPU.

* diag(A) of the assembled A = delta I - E N equals the value formed element by element from
  the interpolation weights: delta - (sum of the cubic weights of the node's own axis
  neighbours that lie in its stencil) / h^2.
* With the plain residual f - A u the cycle's fixed point is the sparse direct solution of
  A u = f (SciPy's spsolve).
* With the residual the paper recommends, f - A(E u), the increments go to zero faster than
  with the plain residual, the residual f - A u stalls (the fixed point is not A u = f), and
  the limit is second-order accurate against the closed-form solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import band as ob
from oracle import standard as os_
from oracle import vcycle as ov


def _hier(cfg):
    return ob.build_hierarchy(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)


@pytest.mark.parametrize("cfg", [W.config_circle(32, 3), W.config_sphere(16, 2)], ids=["circle32", "sphere16"])
def test_diag_from_weights(cfg):
    H = _hier(cfg)
    lev = H.levels[0]
    d = lev.dim
    S = os_.StdHierarchy(H, os_.StdParams())
    base, W1, _ = ob.stencil(lev.cp, lev.h, 3)
    expect = np.full(lev.n, ov.delta(H, 0, 1.0))
    for a in range(d):
        for sgn in (-1, 1):
            nb = lev.idx.copy()
            nb[:, a] += sgn
            rel = nb - base  # position of the neighbour inside the node's stencil box
            inside = np.all((rel >= 0) & (rel <= 3), axis=1)
            w = np.ones(lev.n)
            for b in range(d):
                w *= W1[np.arange(lev.n), b, np.clip(rel[:, b], 0, 3)]
            expect -= np.where(inside, w, 0.0) / lev.h ** 2
    assert np.max(np.abs(S.diag[0] - expect)) <= 1e-12 * np.max(np.abs(expect))
    # the diagonal differs from delta wherever a neighbour falls in the node's own stencil
    assert np.any(np.abs(S.diag[0] - ov.delta(H, 0, 1.0)) > 1.0)


@pytest.mark.parametrize("cfg", [W.config_circle(32, 3), W.config_sphere(12, 2)], ids=["circle32", "sphere12"])
def test_plain_residual_fixed_point_is_sparse_solve(cfg):
    H = _hier(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    res = os_.solve(H, f, os_.StdParams(residual="plain"), rtol=1e-14, max_cycles=120)
    A = os_.matrix_A(H, 0, 1.0)
    u_star = spla.spsolve(A.tocsc(), f)
    assert np.max(np.abs(res.u - u_star)) <= 1e-10 * np.max(np.abs(u_star))
    assert res.residuals[-1] < 1e-11


def test_extended_residual_converges_faster_to_an_accurate_limit():
    cfgs = [W.config_circle(32, 3), W.config_circle(64, 4)]
    errs = []
    for cfg in cfgs:
        H = _hier(cfg)
        cp = H.levels[0].cp
        f = cfg.problem.f(cp)
        ext = os_.solve(H, f, os_.StdParams(), rtol=1e-12, max_cycles=60)
        plain = os_.solve(H, f, os_.StdParams(residual="plain"), rtol=0.0, max_cycles=ext.cycles)
        assert ext.increments[-1] < 1e-12
        assert ext.cycles < 30
        # the paper's observation: the extended residual keeps the cycle contracting faster
        assert ext.increments[9] < 1e-2 * plain.increments[9]
        # ... and its fixed point is not the solution of A u = f
        assert ext.residuals[-1] > 1e-6
        errs.append(np.max(np.abs(ext.u - cfg.problem.u_exact(cp))))
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


def test_extended_residual_sphere():
    cfg = W.config_sphere(16, 2)
    H = _hier(cfg)
    cp = H.levels[0].cp
    f = cfg.problem.f(cp)
    ext = os_.solve(H, f, os_.StdParams(), rtol=1e-11, max_cycles=60)
    assert ext.increments[-1] < 1e-11
    err = np.max(np.abs(ext.u - cfg.problem.u_exact(cp)))
    ref = ov.solve(H, f, ov.Params(), rtol=1e-12, max_cycles=60)
    err_rm = np.max(np.abs(ref.u - cfg.problem.u_exact(cp)))
    # same discretization accuracy as the Ruuth-Merriman solver's limit
    assert err < 2.0 * err_rm and err_rm < 2.0 * err, (err, err_rm)


def test_two_colour_sweep_on_a_red_black_coupled_matrix():
    """On the 1-D Laplacian (red rows couple only to black ones) the red half-sweep with
    omega = 1 zeroes the red rows of the residual exactly, and the black half-sweep then the
    black rows: the textbook red-black Gauss-Seidel step."""
    import scipy.sparse as sp

    n = 41
    A = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    red = (np.arange(n) % 2) == 0
    f = np.random.default_rng(0).standard_normal(n)
    u0 = np.random.default_rng(1).standard_normal(n)
    diag = A.diagonal()
    u_red = u0.copy()
    u_red[red] += (f - A @ u0)[red] / diag[red]
    assert np.max(np.abs((f - A @ u_red)[red])) < 1e-13
    u1 = os_.two_colour_sweep(A, diag, red, u0, f, 1.0)
    assert np.array_equal(u1[red], u_red[red])
    assert np.max(np.abs((f - A @ u1)[~red])) < 1e-13
    # the black half-sweep used the updated red values (Jacobi from u0 would not zero them)
    u_jac = u0 + (f - A @ u0) / diag
    assert np.max(np.abs((f - A @ u_jac)[~red])) > 1e-3


@pytest.mark.parametrize("cfg", [W.config_circle(32, 3), W.config_sphere(12, 2)], ids=["circle32", "sphere12"])
def test_redblack_plain_residual_fixed_point_is_sparse_solve(cfg):
    H = _hier(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    res = os_.solve(H, f, os_.StdParams(residual="plain", smoother="redblack"), rtol=1e-14, max_cycles=120)
    A = os_.matrix_A(H, 0, 1.0)
    u_star = spla.spsolve(A.tocsc(), f)
    assert np.max(np.abs(res.u - u_star)) <= 1e-10 * np.max(np.abs(u_star))


def test_linear_el_operator_vcycle_reaches_table_3_1():
    """Remark 3.2's operator (p = 1 in front of L, q = 3) under the standard-relaxation V-cycle
    with the plain residual: the fixed point is the sparse direct solve of A u = f, and its
    error on the circle reproduces Table 3.1 (dx = 0.025, 0.0125) within 1 %."""
    from oracle import direct as od
    from oracle import errors as oe

    prob = W.circle_sin12()
    table = dict((round(1 / dx), e) for dx, e in [(0.025, 4.76e-3), (0.0125, 1.19e-3)])
    for h_inv, ref in table.items():
        H = ob.build_hierarchy(prob.surface, 1.0 / h_inv, 3, W.LAM2_2D)
        f = prob.f(H.levels[0].cp)
        res = os_.solve(H, f, os_.StdParams(residual="plain", el_degree=1), rtol=1e-13, max_cycles=120)
        A = od.assemble_A(H.levels[0], 1.0, p=1, q=3)
        u_star = spla.spsolve(A.tocsc(), f)
        assert np.max(np.abs(res.u - u_star)) <= 1e-10 * np.max(np.abs(u_star))
        e = oe.surface_error(H.levels[0], res.u, prob.u_exact, 20000)
        assert abs(e - ref) / ref < 0.01, (h_inv, e, ref)
