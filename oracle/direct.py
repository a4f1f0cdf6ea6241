"""Assembled difference scheme and sparse direct solves (Sec. 3.1, eqs. (3.2)-(3.3)).

A^h = c I - M^h,  M^h = E_p L - gamma (I - E_q),  gamma = 2d/h^2 by default.
The direct solve of eq. (3.2) is A^h u = f^h with f^h = f(cp(x_i)) (Sec. 3.4.1).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .band import Level, extension_matrix, laplacian_matrix


def assemble_M(lev: Level, p: int = 3, q: int = 3, gamma: Optional[float] = None) -> sp.csr_matrix:
    d = lev.dim
    if gamma is None:
        gamma = 2.0 * d / (lev.h * lev.h)
    Ep = extension_matrix(lev, p)
    Eq = Ep if q == p else extension_matrix(lev, q)
    L = laplacian_matrix(lev)
    I = sp.identity(lev.n, format="csr")
    return (Ep @ L - gamma * (I - Eq)).tocsr()


def assemble_A(lev: Level, c: float, p: int = 3, q: int = 3, gamma: Optional[float] = None) -> sp.csr_matrix:
    M = assemble_M(lev, p, q, gamma)
    return (c * sp.identity(lev.n, format="csr") - M).tocsr()


def solve_direct(lev: Level, rhs: np.ndarray, c: float, p: int = 3, q: int = 3,
                 gamma: Optional[float] = None) -> np.ndarray:
    A = assemble_A(lev, c, p, q, gamma).tocsc()
    return spla.spsolve(A, rhs)
