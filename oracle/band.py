"""Computational band and discrete operators of the Closest Point Method.

* Band (Sec. 3.1, Fig. 3.1): the grid nodes x = h * i (i integer, grid aligned with the
  origin) whose distance to the surface is at most lambda * h.  lambda^2 = 13 in 2-D and
  17 in 3-D, which contains B_interp (every node of a cubic interpolation stencil of a
  surface point) and B_edge (their Laplacian neighbours).  Table 4.1 pins this rule.
  Nodes are ordered lexicographically with x varying fastest (then y, then z), so the
  four nodes of an interpolation stencil along x are consecutive entries.
* Interpolation (Sec. 3.1): tensor-product Lagrange interpolation of degree p at the
  closest point; per axis the stencil starts at floor(t) - (p - 1)/2 with t = y/h and the
  1-D weights are the Lagrange basis polynomials evaluated in product form
  (closed forms in the proof of Thm 3.4).  All (p+1)^d weights are kept, including exact
  zeros, so nnz(E_3) = 64 n in 3-D (Table 4.1).
* Laplacian (Sec. 3.1): (2d+1)-point centred stencil; neighbours outside the band are
  dropped (the rows of B_edge nodes never reach a closest-point evaluation, eq. (3.2)
  and the remark after it).  N = (sum of in-band neighbours) / h^2, L = N - (2d/h^2) I.
* Restriction / prolongation (Sec. 4.3): closest-point interpolation between the bands of
  two grid levels, linear (degree 1) in the experiments of Sec. 4.6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from workloads import Surface
from .geometry import bounding_box, closest_point_and_dist2


@dataclass
class Level:
    surface: Surface
    h: float
    lam2: float
    idx: np.ndarray  # (n, d) int64 grid multi-indices in band order
    cp: np.ndarray  # (n, d) closest points
    lo: np.ndarray  # (d,) lower corner of the index box
    ext: np.ndarray  # (d,) extents of the index box
    keys: np.ndarray  # (n,) sorted linear keys

    @property
    def n(self) -> int:
        return self.idx.shape[0]

    @property
    def dim(self) -> int:
        return self.idx.shape[1]

    def key_of(self, M: np.ndarray) -> np.ndarray:
        """Linear key of multi-indices M (x fastest); -1 outside the index box."""
        M = np.asarray(M, dtype=np.int64)
        R = M - self.lo
        inside = np.all((R >= 0) & (R < self.ext), axis=1)
        k = np.zeros(M.shape[0], dtype=np.int64)
        mul = 1
        for a in range(self.dim):
            k += R[:, a] * mul
            mul *= int(self.ext[a])
        k[~inside] = -1
        return k

    def lookup(self, M: np.ndarray) -> np.ndarray:
        """Band index of multi-indices M, -1 where the node is not in the band."""
        k = self.key_of(M)
        pos = np.searchsorted(self.keys, k)
        pos = np.minimum(pos, self.n - 1)
        ok = (k >= 0) & (self.keys[pos] == k)
        return np.where(ok, pos, -1)


def build_level(s: Surface, h: float, lam2: float) -> Level:
    """Nodes h*i with dist(h*i, S)^2 <= lam2 * (h*h), in x-fastest lexicographic order."""
    d = s.dim
    lo_b, hi_b = bounding_box(s)
    lam = math.sqrt(lam2)
    ilo = np.floor((lo_b - lam * h) / h).astype(np.int64) - 2
    ihi = np.ceil((hi_b + lam * h) / h).astype(np.int64) + 2
    ext = ihi - ilo + 1
    thr = lam2 * (h * h)
    idx_parts = []
    cp_parts = []
    # enumerate one plane of the slowest axis at a time (bounded memory); inside a plane
    # the nodes come out y-major / x-minor, so concatenating planes gives sorted order
    xs = np.arange(ilo[0], ihi[0] + 1, dtype=np.int64)
    ys = np.arange(ilo[1], ihi[1] + 1, dtype=np.int64)
    if d == 2:
        YY, XX = np.meshgrid(ys, xs, indexing="ij")
        I = np.stack([XX.ravel(), YY.ravel()], axis=1)
        cp, dist2 = closest_point_and_dist2(s, I.astype(np.float64) * h, thr)
        keep = dist2 <= thr
        idx_parts.append(I[keep])
        cp_parts.append(cp[keep])
    else:
        YY, XX = np.meshgrid(ys, xs, indexing="ij")
        XY = np.stack([XX.ravel(), YY.ravel()], axis=1)
        for z in range(ilo[2], ihi[2] + 1):
            I = np.concatenate([XY, np.full((XY.shape[0], 1), z, dtype=np.int64)], axis=1)
            cp, dist2 = closest_point_and_dist2(s, I.astype(np.float64) * h, thr)
            keep = dist2 <= thr
            if keep.any():
                idx_parts.append(I[keep])
                cp_parts.append(cp[keep])
    idx = np.concatenate(idx_parts, axis=0)
    cp = np.concatenate(cp_parts, axis=0)
    lev = Level(s, float(h), float(lam2), idx, cp, ilo, ext, np.empty(0, np.int64))
    lev.keys = lev.key_of(idx)
    assert np.all(np.diff(lev.keys) > 0), "band must come out sorted"
    return lev


def lagrange_weights(s: np.ndarray, p: int) -> np.ndarray:
    """Lagrange basis on nodes 0..p evaluated at s, in product form (exact zeros at nodes)."""
    s = np.asarray(s, dtype=np.float64)
    W = np.ones(s.shape + (p + 1,))
    for j in range(p + 1):
        for k in range(p + 1):
            if k != j:
                W[..., j] *= (s - k) / (j - k)
    return W


def stencil(Y: np.ndarray, h: float, p: int):
    """Degree-p interpolation stencil of points Y on the grid of spacing h.

    Returns (base multi-index (m,d), 1-D weights (m,d,p+1), frac (m,d)) where
    frac = t - floor(t), t = Y/h."""
    t = np.asarray(Y, dtype=np.float64) / h
    fl = np.floor(t)
    frac = t - fl
    base = fl.astype(np.int64) - (p - 1) // 2
    s = frac + (p - 1) // 2
    return base, lagrange_weights(s, p), frac


def stencil_offsets(d: int, p: int) -> np.ndarray:
    """Offsets of a (p+1)^d stencil, x fastest."""
    r = np.arange(p + 1)
    if d == 2:
        B, A = np.meshgrid(r, r, indexing="ij")
        return np.stack([A.ravel(), B.ravel()], axis=1)
    C, B, A = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([A.ravel(), B.ravel(), C.ravel()], axis=1)


def tensor_weights(W1: np.ndarray) -> np.ndarray:
    """(m,d,p+1) 1-D weights -> (m,(p+1)^d) tensor weights, x fastest."""
    m, d, q = W1.shape
    if d == 2:
        return (W1[:, 1, :, None] * W1[:, 0, None, :]).reshape(m, q * q)
    return (W1[:, 2, :, None, None] * W1[:, 1, None, :, None] * W1[:, 0, None, None, :]).reshape(m, q ** 3)


def interp_matrix(Y: np.ndarray, target: Level, p: int, rows: Optional[int] = None) -> sp.csr_matrix:
    """Matrix evaluating the degree-p interpolant of band values of ``target`` at points Y.

    Raises if a stencil node is missing from the band."""
    m, d = Y.shape
    base, W1, _ = stencil(Y, target.h, p)
    off = stencil_offsets(d, p)
    M = base[:, None, :] + off[None, :, :]
    cols = target.lookup(M.reshape(-1, d)).reshape(m, -1)
    if np.any(cols < 0):
        bad = int(np.argmax(np.any(cols < 0, axis=1)))
        raise ValueError("interpolation stencil leaves the band (point %d, h=%g)" % (bad, target.h))
    vals = tensor_weights(W1)
    q = off.shape[0]
    indptr = np.arange(0, m * q + 1, q)
    return sp.csr_matrix((vals.ravel(), cols.ravel(), indptr), shape=(m, target.n))


def extension_matrix(lev: Level, p: int = 3) -> sp.csr_matrix:
    """E_p: degree-p closest-point interpolation at cp(x_i) for every band node (eq. (3.2))."""
    return interp_matrix(lev.cp, lev, p)


def neighbour_indices(lev: Level) -> np.ndarray:
    """(n, 2d) band indices of the -x,+x,-y,+y(,-z,+z) neighbours, -1 if absent."""
    d = lev.dim
    out = np.empty((lev.n, 2 * d), dtype=np.int64)
    for a in range(d):
        for sgn_i, sgn in enumerate((-1, 1)):
            M = lev.idx.copy()
            M[:, a] += sgn
            out[:, 2 * a + sgn_i] = lev.lookup(M)
    return out


def neighbour_sum_matrix(lev: Level) -> sp.csr_matrix:
    """N = (sum over in-band axis neighbours)/h^2; L = N - (2d/h^2) I (Sec. 3.1)."""
    nb = neighbour_indices(lev)
    rows = np.repeat(np.arange(lev.n), nb.shape[1])
    cols = nb.ravel()
    ok = cols >= 0
    vals = np.full(ok.sum(), 1.0 / (lev.h * lev.h))
    return sp.csr_matrix((vals, (rows[ok], cols[ok])), shape=(lev.n, lev.n))


def laplacian_matrix(lev: Level) -> sp.csr_matrix:
    d = lev.dim
    return (neighbour_sum_matrix(lev) - (2.0 * d / (lev.h * lev.h)) * sp.identity(lev.n, format="csr")).tocsr()


def check_containment(lev: Level, E: sp.csr_matrix) -> None:
    """Every node of an interpolation stencil must have all of its Laplacian neighbours in
    the band (B_interp and B_edge both inside B, Sec. 3.1)."""
    used = np.unique(E.indices)
    nb = neighbour_indices(lev)[used]
    if np.any(nb < 0):
        raise ValueError("band too narrow: a stencil node lacks a Laplacian neighbour (h=%g)" % lev.h)


def restriction_matrix(fine: Level, coarse: Level, p: int = 1) -> sp.csr_matrix:
    """E_h^{2h}: value at a coarse node = interpolation at its closest point of fine-band values."""
    return interp_matrix(coarse.cp, fine, p)


def prolongation_matrix(fine: Level, coarse: Level, p: int = 1) -> sp.csr_matrix:
    """E_{2h}^h: value at a fine node = interpolation at its closest point of coarse-band values."""
    return interp_matrix(fine.cp, coarse, p)


@dataclass
class Hierarchy:
    levels: List[Level]
    E: List[sp.csr_matrix]
    N: List[sp.csr_matrix]
    R: List[sp.csr_matrix]  # R[l]: level l -> l+1
    P: List[sp.csr_matrix]  # P[l]: level l+1 -> l


def build_hierarchy(s: Surface, h0: float, nlev: int, lam2: float,
                    interp_degree: int = 3, transfer_degree: int = 1) -> Hierarchy:
    """Bands on h_l = h0 * 2^l, l = 0..nlev-1, each with its own tube of radius lambda*h_l
    (Sec. 4.3: the coarse band is wider than the fine one)."""
    levels = [build_level(s, h0 * (2 ** l), lam2) for l in range(nlev)]
    E, N, R, P = [], [], [], []
    for l, lev in enumerate(levels):
        El = extension_matrix(lev, interp_degree)
        check_containment(lev, El)
        E.append(El)
        N.append(neighbour_sum_matrix(lev))
    for l in range(nlev - 1):
        R.append(restriction_matrix(levels[l], levels[l + 1], transfer_degree))
        P.append(prolongation_matrix(levels[l], levels[l + 1], transfer_degree))
    return Hierarchy(levels, E, N, R, P)
