"""Variable diffusion coefficients: -div_S(a grad_S u) + c u = f (Sec. 2.2; the
variable-coefficient sphere example, Sec. 4.6.6).

Discretization (as the paper writes it): L~ = sum over axes of D^b diag(A^f a) D^f, with
a_i = a(cp(x_i)), D^f / D^b forward / backward differences and A^f the average of two
neighbouring values of a along the positive axis.  At node j this is

    L~ u_j = sum_axes [ abar_j+ (u_j+ - u_j) - abar_j- (u_j - u_j-) ] / h^2,
    abar_j+- = (a_j + a_j+-) / 2,

split here as L~ = N~ - diag(sigma): N~ the weighted neighbour sum, sigma_j = sum of the
abar of node j / h^2.  Neighbours outside the band are dropped from N~, as for L (only rows
of stencil nodes are ever used, and all their neighbours are in the band); in sigma a
missing neighbour counts with the node's own a, so that for a = 1 the diagonal is the
2d/h^2 of L on every row, edge rows included.

Smoothing (the paper keeps the Ruuth-Merriman strategy with L replaced by L~): one Jacobi
step on A~ = cI - L~, u~ = u + (f - A~ u) / (c + sigma) = (f + N~ u) / (c + sigma), then the
extension, u <- (1 - omega) u + omega E u~.

Residual and coarsest solve (a reading; the paper does not spell them out): the smoother's
fixed point satisfies u = E D^{-1} (f + N~ u), D = diag(c + sigma), i.e.
(I - E D^{-1} N~) u = E D^{-1} f.  The residual of a level is that equation's residual
brought to the units of f node by node: r = D (E u~ - u) with u~ the undamped Jacobi step
(for a = 1, D = delta and it is the residual of the constant-coefficient cycle exactly).
The coarse level then solves (I - E_c D_c^{-1} N~_c) e = E_c D_c^{-1} R r, whose right-hand
side carries the ratio D / D_c of the two levels' diagonals at every node; a level-constant
scale in place of D would be off by the factor a and lets the cycle diverge for a variable
coefficient.  The coarsest level solves its fixed-point equation directly.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .band import Hierarchy, Level, neighbour_indices


def flux_operator(lev: Level, a: np.ndarray):
    """(N~ as CSR, sigma) of L~ = N~ - diag(sigma) on one level, a = a(cp(x)) per node."""
    nb = neighbour_indices(lev)
    n = lev.n
    ih2 = 1.0 / (lev.h * lev.h)
    rows, cols, vals = [], [], []
    sigma = np.zeros(n)
    for q in range(nb.shape[1]):
        j = nb[:, q]
        ok = j >= 0
        abar = a.astype(np.float64).copy()  # missing neighbour: a_j itself
        abar[ok] = 0.5 * (a[ok] + a[j[ok]])
        rows.append(np.nonzero(ok)[0])
        cols.append(j[ok])
        vals.append(abar[ok] * ih2)
        sigma += abar * ih2
    Nt = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return Nt, sigma


@dataclass
class VCParams:
    c: float = 1.0
    nu1: int = 3
    nu2: int = 3
    omega: float = 2.0 / 3.0


class VCHierarchy:
    def __init__(self, H: Hierarchy, a_levels: List[np.ndarray], p: VCParams):
        self.H = H
        self.p = p
        self.Nt, self.D = [], []
        for lev, a in zip(H.levels, a_levels):
            Nt, sigma = flux_operator(lev, a)
            self.Nt.append(Nt)
            self.D.append(p.c + sigma)
        l = len(H.levels) - 1
        n = H.levels[l].n
        Ec = H.E[l]
        Mc = sp.identity(n, format="csr") - Ec @ sp.diags(1.0 / self.D[l]) @ self.Nt[l]
        self.lu = sla.lu_factor(Mc.toarray())


def jacobi_step(S: VCHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """u~ = (f + N~ u) / (c + sigma): one undamped Jacobi step on A~ = cI - L~."""
    return (f + S.Nt[l] @ u) / S.D[l]


def smooth(S: VCHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    om = S.p.omega
    return (1.0 - om) * u + om * (S.H.E[l] @ jacobi_step(S, l, u, f))


def residual(S: VCHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    return S.D[l] * (S.H.E[l] @ jacobi_step(S, l, u, f) - u)


def vcycle(S: VCHierarchy, l: int, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    H = S.H
    if l == len(H.levels) - 1:
        return sla.lu_solve(S.lu, H.E[l] @ (f / S.D[l]))
    for _ in range(S.p.nu1):
        u = smooth(S, l, u, f)
    ec = vcycle(S, l + 1, np.zeros(H.levels[l + 1].n), H.R[l] @ residual(S, l, u, f))
    u = u + H.P[l] @ ec
    for _ in range(S.p.nu2):
        u = smooth(S, l, u, f)
    return u


@dataclass
class VCResult:
    u: np.ndarray
    relres: List[float]  # ||r(u_k)||_inf / ||D E D^{-1} f||_inf
    iterates: List[np.ndarray]

    @property
    def cycles(self) -> int:
        return len(self.relres)


def rhs_norm(S: VCHierarchy, f: np.ndarray) -> float:
    return float(np.max(np.abs(S.D[0] * (S.H.E[0] @ (f / S.D[0])))))


def solve(H: Hierarchy, a_levels: List[np.ndarray], f: np.ndarray, p: VCParams, rtol: float = 1e-10,
          max_cycles: int = 60, keep_iterates: bool = False) -> VCResult:
    S = VCHierarchy(H, a_levels, p)
    u = np.zeros(H.levels[0].n)
    bn = rhs_norm(S, f)
    res, its = [], []
    for _ in range(max_cycles):
        u = vcycle(S, 0, u, f)
        res.append(float(np.max(np.abs(residual(S, 0, u, f)))) / bn)
        if keep_iterates:
            its.append(u.copy())
        if res[-1] < rtol:
            break
    return VCResult(u, res, its)


def fixed_point(H: Hierarchy, a_levels: List[np.ndarray], f: np.ndarray, p: VCParams) -> np.ndarray:
    """Sparse direct solve of the fine level's fixed-point equation (I - E D^{-1} N~) u = E D^{-1} f."""
    import scipy.sparse.linalg as spla

    S = VCHierarchy(H, a_levels, p)
    n = H.levels[0].n
    M = sp.identity(n, format="csc") - (H.E[0] @ sp.diags(1.0 / S.D[0]) @ S.Nt[0]).tocsc()
    return spla.spsolve(M, H.E[0] @ (f / S.D[0]))
