"""The V-cycle with standard relaxation (Sec. 4.5), on the same bands and transfers.

Instead of the Ruuth-Merriman step (Jacobi on A~ followed by an extension, Sec. 4.2),
steps 1 and 4 of Algorithm 4.1 apply the Jacobi iteration of Sec. 4.1 to the linear
system A u = f of eq. (3.3) itself:

    u <- u + omega diag(A)^{-1} (f - A u),      A = cI - M = delta I - E N,

(the paper's iteration is undamped, omega = 1; the damping factor is the same parameter as
for the Ruuth-Merriman smoother).  The residual passed to the coarse grid is the one the
paper recommends with this smoother, r = f - A (E u) (``residual="extended"``); the plain
residual r = f - A u is kept as ``residual="plain"``.  Every level solves for a correction
of its own system A_l e = f_l (f-space right-hand sides, no extension in front of them),
and the coarsest level is solved exactly, e = A_c^{-1} f_c.

The operator may also be the sparser one of Remark 3.2, A = c I - (E_1 L - gamma (I - E_3))
with linear interpolation in front of the Laplacian (``el_degree=1``), which the paper uses
for its direct solves (Table 3.1); the extended residual keeps the cubic E.

The stopping test is the paper's (Sec. 4.6): the relative increment
||u_{k+1} - u_k||_inf / ||u_{k+1}||_inf.  With the extended residual the cycle's fixed point
is not the solution of A u = f (the residual f - A u stalls at the size of the
discretization error while the increments go to zero); with the plain residual it is.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .band import Hierarchy
from .direct import assemble_A
from .vcycle import delta


@dataclass
class StdParams:
    c: float = 1.0
    nu1: int = 3
    nu2: int = 3
    omega: float = 2.0 / 3.0
    residual: str = "extended"  # r = f - A (E u); "plain": r = f - A u
    gamma: int = 1  # cycle index (1: V-cycle, 2: W-cycle)
    smoother: str = "jacobi"  # or "redblack": two-colour Gauss-Seidel ordering of the same step
    el_degree: int = 3  # degree p of the interpolation in front of L (1: Remark 3.2's sparser M)


def matrix_A(H: Hierarchy, l: int, c: float, el_degree: int = 3) -> sp.csr_matrix:
    """A = c I - M on level l, M = E_p L - gamma (I - E_3) (eq. (3.3)); with p = 3 this is
    delta I - E N.  p = 1 is the sparser operator of Remark 3.2 (linear interpolation in front
    of the Laplacian, the one of Table 3.1), assembled by the direct-solve module."""
    if el_degree == 1:
        return assemble_A(H.levels[l], c, p=1, q=3)
    n = H.levels[l].n
    return (delta(H, l, c) * sp.identity(n, format="csr") - H.E[l] @ H.N[l]).tocsr()


def red_nodes(lev) -> np.ndarray:
    """Colour of the two-colour ordering: nodes whose grid indices sum to an even number."""
    return (np.sum(lev.idx, axis=1) % 2) == 0


class StdHierarchy:
    """The assembled A_l, their diagonals, node colours and the LU factors of the coarsest A_c."""

    def __init__(self, H: Hierarchy, p: StdParams):
        self.H = H
        self.p = p
        self.A = [matrix_A(H, l, p.c, p.el_degree) for l in range(len(H.levels))]
        self.diag = [A.diagonal() for A in self.A]
        self.red = [red_nodes(lev) for lev in H.levels]
        self.lu = sla.lu_factor(self.A[-1].toarray())


def two_colour_sweep(A, diag: np.ndarray, red: np.ndarray, u: np.ndarray, f: np.ndarray,
                     omega: float) -> np.ndarray:
    """Gauss-Seidel in two-colour (red-black) order: the damped Jacobi correction
    omega (f - A u) / diag(A) applied to the red rows from the current iterate, then to the
    black rows from the iterate the red half-sweep left (Sec. 4.5 names Gauss-Seidel as an
    alternative to Jacobi).  Rows of one colour that couple to each other (A = delta I - E N
    couples a node to the nodes of its stencil) are updated together, as Jacobi does."""
    u = u.copy()
    for colour in (red, ~red):
        r = f - A @ u
        u[colour] += omega * r[colour] / diag[colour]
    return u


def smooth(S: StdHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """One damped Jacobi step on A_l u = f (Sec. 4.1, the iteration of Sec. 4.5), or one
    red-black Gauss-Seidel sweep of it."""
    if S.p.smoother == "redblack":
        return two_colour_sweep(S.A[l], S.diag[l], S.red[l], u, f, S.p.omega)
    return u + S.p.omega * (f - S.A[l] @ u) / S.diag[l]


def residual(S: StdHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    if S.p.residual == "plain":
        return f - S.A[l] @ u
    return f - S.A[l] @ (S.H.E[l] @ u)


def vcycle(S: StdHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Algorithm 4.1 with the standard relaxation in steps 1 and 4."""
    H = S.H
    if l == len(H.levels) - 1:
        return sla.lu_solve(S.lu, f)
    for _ in range(S.p.nu1):
        u = smooth(S, l, u, f)
    fc = H.R[l] @ residual(S, l, u, f)
    ec = np.zeros(H.levels[l + 1].n)
    for _ in range(1 if l + 1 == len(H.levels) - 1 else max(1, S.p.gamma)):
        ec = vcycle(S, l + 1, ec, fc)
    u = u + H.P[l] @ ec
    for _ in range(S.p.nu2):
        u = smooth(S, l, u, f)
    return u


@dataclass
class StdResult:
    u: np.ndarray
    increments: List[float]  # ||u_k - u_{k-1}||_inf / ||u_k||_inf after each cycle
    residuals: List[float]  # ||f - A u_k||_inf / ||f||_inf
    iterates: Optional[List[np.ndarray]] = None

    @property
    def cycles(self) -> int:
        return len(self.increments)


def solve(H: Hierarchy, f: np.ndarray, p: StdParams, rtol: float = 1e-10, max_cycles: int = 60,
          keep_iterates: bool = False) -> StdResult:
    """V-cycles from u_0 = 0 until the relative increment drops below rtol."""
    S = StdHierarchy(H, p)
    u = np.zeros(H.levels[0].n)
    fn = float(np.max(np.abs(f)))
    inc, res, its = [], [], []
    for _ in range(max_cycles):
        un = vcycle(S, 0, u, f)
        inc.append(float(np.max(np.abs(un - u))) / max(float(np.max(np.abs(un))), 1e-300))
        u = un
        res.append(float(np.max(np.abs(f - S.A[0] @ u))) / fn)
        if keep_iterates:
            its.append(u.copy())
        if inc[-1] < rtol:
            break
    return StdResult(u, inc, res, its if keep_iterates else None)
