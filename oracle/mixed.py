"""Mixed-precision iterative refinement around the CPM V-cycle.

The paper runs everything in double precision (MATLAB).  This variant keeps double
precision only where the fixed point is decided: the outer residual r = E f - A u
(eq. (3.3)), the update u += e and the coarsest direct solve; the inner V-cycle
(smoothing, extension, restriction, prolongation) runs in float32.

The inner V-cycle solves the correction equation A e = r.  Because the damped
Ruuth-Merriman step equals e <- e + (omega/delta)(b - A e) with b = E f, the same
smoother applied to an arbitrary right-hand side b in "A-space" reads
e <- (1 - omega) e + (omega/delta)(b + E N e).  The finest level of the inner cycle
uses that form with b = r; coarser levels keep the f-space form of Algorithm 4.1
(the restricted residual is extended by E before use).  In exact arithmetic one outer
step therefore equals one double-precision V-cycle, so the contraction per step is the
same and the refinement converges to the double-precision fixed point A^{-1} E f.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .band import Hierarchy
from .vcycle import Params, SolveResult, coarse_matrix, delta, rhs_norm


class _H32:
    def __init__(self, H: Hierarchy):
        f32 = np.float32
        self.E = [m.astype(f32) for m in H.E]
        self.N = [m.astype(f32) for m in H.N]
        self.R = [m.astype(f32) for m in H.R]
        self.P = [m.astype(f32) for m in H.P]
        self.levels = H.levels


def _vcycle32(H32: _H32, H: Hierarchy, l: int, e: np.ndarray, rhs: np.ndarray, aspace: bool,
              p: Params, lu) -> np.ndarray:
    f32 = np.float32
    last = len(H.levels) - 1
    if l == last:
        # coarsest solve in double precision: A_c e = E_c f_c
        rhs64 = H.E[l] @ rhs.astype(np.float64)
        return sla.lu_solve(lu, rhs64).astype(f32)
    dl = f32(delta(H, l, p.c))
    w = f32(p.omega)
    one = f32(1.0)

    def ext(u):
        if aspace:
            return rhs + H32.E[l] @ (H32.N[l] @ u)
        return H32.E[l] @ (rhs + H32.N[l] @ u)

    for _ in range(p.nu1):
        e = (one - w) * e + w * ext(e) / dl
    r = ext(e) - dl * e
    fc = H32.R[l] @ r
    ec = _vcycle32(H32, H, l + 1, np.zeros(H.levels[l + 1].n, f32), fc, False, p, lu)
    e = e + H32.P[l] @ ec
    for _ in range(p.nu2):
        e = (one - w) * e + w * ext(e) / dl
    return e


def solve_mixed(H: Hierarchy, f: np.ndarray, p: Params, rtol: float = 1e-10,
                max_cycles: int = 60, u0: Optional[np.ndarray] = None) -> SolveResult:
    """Outer loop in float64, one float32 V-cycle per outer step (A-space RHS on level 0),
    from u0 (default 0; e.g. the float64 full-multigrid start of vcycle.fmg_start)."""
    H32 = _H32(H)
    lu = sla.lu_factor(coarse_matrix(H, p.c))
    d0 = delta(H, 0, p.c)
    bn = rhs_norm(H, f)
    u = np.zeros(H.levels[0].n) if u0 is None else np.array(u0, dtype=np.float64)
    res: List[float] = []
    inc: List[float] = []
    r = H.E[0] @ (f + H.N[0] @ u) - d0 * u
    for _ in range(max_cycles):
        e = _vcycle32(H32, H, 0, np.zeros(H.levels[0].n, np.float32), r.astype(np.float32), True, p, lu)
        u = u + e.astype(np.float64)
        inc.append(float(np.max(np.abs(e))) / max(float(np.max(np.abs(u))), 1e-300))
        r = H.E[0] @ (f + H.N[0] @ u) - d0 * u
        res.append(float(np.max(np.abs(r))) / bn)
        if res[-1] < rtol:
            break
    return SolveResult(u, res, inc)
