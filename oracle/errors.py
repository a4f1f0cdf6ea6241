"""Error of a band solution against a closed-form surface solution (Sec. 3.4.1):
either at the grid nodes against u(cp(x_i)), or at many sample points on the surface
after cubic interpolation of the band values."""
from __future__ import annotations

import math

import numpy as np

from workloads import CIRCLE, SPHERE, TORUS, Surface
from .band import Level, interp_matrix


def grid_error(lev: Level, u: np.ndarray, u_exact) -> float:
    ue = u_exact(lev.cp)
    return float(np.max(np.abs(u - ue)) / np.max(np.abs(ue)))


def surface_samples(s: Surface, m: int) -> np.ndarray:
    """m points on the surface: uniform angles (circle), Fibonacci lattice (sphere),
    a square (theta, phi) lattice (torus)."""
    c = s.c0()
    if s.kind == CIRCLE:
        t = 2.0 * math.pi * np.arange(m) / m
        return c + s.R * np.stack([np.cos(t), np.sin(t)], axis=1)
    if s.kind == SPHERE:
        k = np.arange(m) + 0.5
        z = 1.0 - 2.0 * k / m
        th = math.pi * (1.0 + 5.0 ** 0.5) * k
        rr = np.sqrt(1.0 - z * z)
        return c + s.R * np.stack([rr * np.cos(th), rr * np.sin(th), z], axis=1)
    q = int(math.ceil(math.sqrt(m)))
    th, ph = np.meshgrid(2 * math.pi * np.arange(q) / q, 2 * math.pi * np.arange(q) / q, indexing="ij")
    th, ph = th.ravel(), ph.ravel()
    rad = s.R + s.r * np.cos(ph)
    return c + np.stack([rad * np.cos(th), rad * np.sin(th), s.r * np.sin(ph)], axis=1)


def surface_error(lev: Level, u: np.ndarray, u_exact, m: int = 20000) -> float:
    Y = surface_samples(lev.surface, m)
    ui = interp_matrix(Y, lev, 3) @ u
    ue = u_exact(Y)
    return float(np.max(np.abs(ui - ue)) / np.max(np.abs(ue)))
