"""Closest Point Method V-cycle (Algorithm 4.1) with Ruuth-Merriman Jacobi smoothing.

Notation per level: N = neighbour sum / h^2 (so L = N - (2d/h^2) I), E = cubic
closest-point interpolation, delta = c + 2d/h^2 = diag(A~) with A~ = cI - L.

* Smoothing (eqs. (4.2a), (4.2b)): one Jacobi step on A~ followed by closest-point
  extension.  Since u + (f - A~ u)/delta = (f + N u)/delta, the step is
  S(u) = E (f + N u) / delta.  A damping factor omega is applied outside the
  extension: u <- (1 - omega) u + omega S(u) (omega = 1 is the paper's step).
* Residual and stopping: the fixed point of the smoother satisfies
  E (f + N u) = delta u, i.e. A u = E f with A = cI - M, M = E L - gamma (I - E),
  gamma = 2d/h^2 (eq. (3.3) with p = q = 3).  The residual passed to the coarse grid and
  used for stopping is therefore r = E (f + N u) - delta u = E f - A u.  Step 2 of
  Algorithm 4.1 prints r = f - A~ u, whose norm stalls at the size of the extension's
  discretization error (Sec. 4.6.1 says so); that literal variant is kept as
  ``residual_mode="verbatim"``.
* Restriction / prolongation: closest-point interpolation between levels (Sec. 4.3).
* Coarsest level: a direct solve, of A_c e = E_c f_c (consistent reading) or of
  A_c e = f_c (verbatim), by dense LU.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .band import Hierarchy


@dataclass
class Params:
    c: float = 1.0
    nu1: int = 3
    nu2: int = 3
    omega: float = 2.0 / 3.0
    residual_mode: str = "consistent"  # or "verbatim"
    learned: Optional[np.ndarray] = None  # bf16 weights of the learned smoother (levels 0, 1)
    learned_sweeps: int = 0  # sweeps per side on the learned levels (0: nu1 / nu2)
    gamma: int = 1  # cycle index: coarse-grid visits per level (1: V-cycle, 2: W-cycle)


def delta(H: Hierarchy, l: int, c: float) -> float:
    lev = H.levels[l]
    return c + 2.0 * lev.dim / (lev.h * lev.h)


def smooth(H: Hierarchy, l: int, u: np.ndarray, f: np.ndarray, p: Params) -> np.ndarray:
    """Damped Ruuth-Merriman Jacobi step: u <- (1-w) u + w E(f + N u)/delta; on the two
    finest levels the learned local step replaces it when weights are given."""
    dl = delta(H, l, p.c)
    if p.learned is not None and l < 2:
        from .mlp import learned_update

        return u + learned_update(H.levels[l], residual(H, l, u, f, p), dl, p.learned)
    g = f + H.N[l] @ u
    return (1.0 - p.omega) * u + p.omega * (H.E[l] @ g) / dl


def residual(H: Hierarchy, l: int, u: np.ndarray, f: np.ndarray, p: Params) -> np.ndarray:
    """r = E(f + N u) - delta u  (= E f - A u); verbatim: r = f - A~ u = f + N u - delta u."""
    dl = delta(H, l, p.c)
    g = f + H.N[l] @ u
    if p.residual_mode == "verbatim":
        return g - dl * u
    return H.E[l] @ g - dl * u


def coarse_matrix(H: Hierarchy, c: float) -> np.ndarray:
    """Dense A_c = delta I - E_c N_c on the coarsest level."""
    l = len(H.levels) - 1
    dl = delta(H, l, c)
    A = -(H.E[l] @ H.N[l]).toarray()
    A[np.diag_indices_from(A)] += dl
    return A


class CoarseSolver:
    def __init__(self, H: Hierarchy, p: Params):
        self.H = H
        self.p = p
        self.l = len(H.levels) - 1
        self.lu = sla.lu_factor(coarse_matrix(H, p.c))

    def __call__(self, fc: np.ndarray) -> np.ndarray:
        rhs = fc if self.p.residual_mode == "verbatim" else self.H.E[self.l] @ fc
        return sla.lu_solve(self.lu, rhs)


def vcycle(H: Hierarchy, l: int, u: np.ndarray, f: np.ndarray, p: Params,
           coarse: CoarseSolver) -> np.ndarray:
    """u^h = V^h(u^h, f^h), Algorithm 4.1, recursing down to the coarsest level."""
    if l == len(H.levels) - 1:
        return coarse(f)
    nu1, nu2 = p.nu1, p.nu2
    if p.learned is not None and l < 2 and p.learned_sweeps > 0:
        nu1 = nu2 = p.learned_sweeps
    for _ in range(nu1):  # step 1: pre-smoothing
        u = smooth(H, l, u, f, p)
    r = residual(H, l, u, f, p)  # step 2: residual, restriction, coarse solve
    fc = H.R[l] @ r
    ec = np.zeros(H.levels[l + 1].n)
    # gamma recursive visits of the coarse level (the coarsest one is solved exactly once)
    for _ in range(1 if l + 1 == len(H.levels) - 1 else max(1, p.gamma)):
        ec = vcycle(H, l + 1, ec, fc, p, coarse)
    u = u + H.P[l] @ ec  # step 3: coarse-grid correction
    for _ in range(nu2):  # step 4: post-smoothing
        u = smooth(H, l, u, f, p)
    return u


@dataclass
class SolveResult:
    u: np.ndarray
    relres: List[float]  # ||E f - A u_k||_inf / ||E f||_inf after each cycle
    increments: List[float]  # ||u_k - u_{k-1}||_inf / ||u_k||_inf (the paper's criterion)
    iterates: Optional[List[np.ndarray]] = None

    @property
    def cycles(self) -> int:
        return len(self.relres)


def rhs_norm(H: Hierarchy, f: np.ndarray) -> float:
    return float(np.max(np.abs(H.E[0] @ f)))


def fmg_start(H: Hierarchy, f: np.ndarray, p: Params, coarse: CoarseSolver) -> np.ndarray:
    """Full-multigrid start (nested iteration): the right-hand side restricted to every level
    with the closest-point restriction, the coarsest level solved exactly, then on each finer
    level the coarse solution interpolated to the fine closest points and improved by one
    cycle.  The nested-iteration interpolation is cubic (degree 3 closest-point
    interpolation): with the cycle's linear prolongation the start misses the discretization
    error by one to three orders of magnitude, with cubic it lands within a small factor of
    it (the classical full-multigrid property)."""
    from .band import interp_matrix

    L = len(H.levels)
    fs = [f]
    for l in range(L - 1):
        fs.append(H.R[l] @ fs[-1])
    u = coarse(fs[L - 1])
    for l in range(L - 2, -1, -1):
        u = vcycle(H, l, interp_matrix(H.levels[l].cp, H.levels[l + 1], 3) @ u, fs[l], p, coarse)
    return u


def solve(H: Hierarchy, f: np.ndarray, p: Params, rtol: float = 1e-10, max_cycles: int = 60,
          keep_iterates: bool = False, u0: Optional[np.ndarray] = None, fmg: bool = False) -> SolveResult:
    """Repeat V-cycles from u_0 = 0 until ||E f - A u||_inf / ||E f||_inf < rtol.

    In verbatim mode the residual of A u = f is reported instead and the loop stops on
    the paper's increment criterion ||u_{k+1} - u_k||_inf / ||u_k||_inf < rtol."""
    coarse = CoarseSolver(H, p)
    u = np.zeros(H.levels[0].n) if u0 is None else u0.copy()
    consistent = Params(p.c, p.nu1, p.nu2, p.omega, "consistent")
    if u0 is None and fmg:
        u = fmg_start(H, f, p, coarse)
    bn = rhs_norm(H, f)
    res, inc, its = [], [], []
    for _ in range(max_cycles):
        un = vcycle(H, 0, u, f, p, coarse)
        du = float(np.max(np.abs(un - u))) / max(float(np.max(np.abs(un))), 1e-300)
        u = un
        r = residual(H, 0, u, f, consistent)
        res.append(float(np.max(np.abs(r))) / bn)
        inc.append(du)
        if keep_iterates:
            its.append(u.copy())
        crit = inc[-1] if p.residual_mode == "verbatim" else res[-1]
        if crit < rtol:
            break
    return SolveResult(u, res, inc, its if keep_iterates else None)


def contraction(relres: List[float], skip: int = 2) -> float:
    """Geometric-mean residual reduction per cycle, ignoring the first ``skip`` cycles."""
    r = np.asarray(relres)
    if len(r) <= skip + 1:
        return float(r[-1] / r[0]) ** (1.0 / max(1, len(r) - 1))
    return float((r[-1] / r[skip]) ** (1.0 / (len(r) - 1 - skip)))
