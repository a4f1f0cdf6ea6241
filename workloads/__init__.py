"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module describes *problems*, never the method: a surface is given by its
kind and parameters, a right-hand side by a closed-form function evaluated at
points that already lie on the surface, and random draws (mode amplitudes,
phases, radii, grid spacings) by a seeded NumPy generator.  Nothing here builds a
band, evaluates a closest point, interpolates or smooths; both the oracle and the
GPU library do that themselves from these descriptions.

Manufactured solutions follow the paper's numerical examples:

* unit circle, u = sin(theta) + sin(12 theta)            (Sec. 3.4.1 / 4.6.1)
* unit sphere, u proportional to Re Y_3^2 (l = 3)        (sphere example of Sec. 4.6,
  here with an l = 3 harmonic) and the paper's l = 5 harmonic cos(3 theta) sin^3(phi)
  (9 cos^2(phi) - 1); for that one the printed right-hand side "-29u" is a misprint:
  an l = 5 harmonic has -Lap_S u = 30 u, so with c = 1 the right-hand side is 31 u
* torus R = 1.2, r = 0.6, u = sin(3 theta) + cos(2 phi) with the closed-form f of the
  torus example of Sec. 4.6
* seeded random mode mixes on tori (16 Fourier modes, mean zero) and spheres
  (real spherical harmonics of degree 1..4, with the exact solution known)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

CIRCLE = "circle"
SPHERE = "sphere"
TORUS = "torus"
DZIUK = "dziuk"  # the level set (x1 - x3^2)^2 + x2^2 + x3^2 = 1 (Dziuk's surface)

#: seed base for the random right-hand sides and batched problem draws
SEED_BASE = 13074354


@dataclass(frozen=True)
class Surface:
    """A closed curve (2-D) or surface (3-D) described by its kind and size.

    circle: centre (cx, cy), radius R.            (embedding dimension 2)
    sphere: centre (cx, cy, cz), radius R.        (embedding dimension 3)
    torus:  centre (cx, cy, cz), axis along z, tube-centre radius R, tube radius r.
    dziuk:  centre (cx, cy, cz) shifts the level set (x1 - x3^2)^2 + x2^2 + x3^2 = 1 (R, r unused).
    """

    kind: str
    R: float
    r: float = 0.0
    center: Tuple[float, ...] = (0.0, 0.0, 0.0)

    @property
    def dim(self) -> int:
        return 2 if self.kind == CIRCLE else 3

    def c0(self) -> np.ndarray:
        return np.asarray(self.center[: self.dim], dtype=np.float64)


def unit_circle() -> Surface:
    return Surface(CIRCLE, 1.0, 0.0, (0.0, 0.0))


def unit_sphere() -> Surface:
    return Surface(SPHERE, 1.0, 0.0, (0.0, 0.0, 0.0))


def torus(R: float, r: float) -> Surface:
    return Surface(TORUS, float(R), float(r), (0.0, 0.0, 0.0))


def dziuk_surface() -> Surface:
    return Surface(DZIUK, 1.0, 0.0, (0.0, 0.0, 0.0))


# ----------------------------------------------------------------------------
# angles of surface points (used only to evaluate closed-form data on S)
# ----------------------------------------------------------------------------

def _theta(Y: np.ndarray, s: Surface) -> np.ndarray:
    c = s.c0()
    return np.arctan2(Y[:, 1] - c[1], Y[:, 0] - c[0])


def _sphere_dirs(Y: np.ndarray, s: Surface) -> np.ndarray:
    c = s.c0()
    return (Y - c) / s.R


def _torus_angles(Y: np.ndarray, s: Surface):
    c = s.c0()
    X = Y - c
    theta = np.arctan2(X[:, 1], X[:, 0])
    rho = np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2)
    phi = np.arctan2(X[:, 2], rho - s.R)
    return theta, phi


# ----------------------------------------------------------------------------
# manufactured problems: u (exact, may be None) and f, both functions of points Y on S
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """-Lap_S u + c u = f on a surface; ``u_exact`` is None when no closed form exists."""

    surface: Surface
    c: float
    f: Callable[[np.ndarray], np.ndarray]
    u_exact: Optional[Callable[[np.ndarray], np.ndarray]]
    name: str = ""
    # scalar diffusion coefficient a(y) of -div_S(a grad_S u) + c u = f (None: a = 1)
    a: Optional[Callable[[np.ndarray], np.ndarray]] = None


def circle_sin12(c: float = 1.0) -> Problem:
    """Unit circle, u = sin(theta) + sin(12 theta); -Lap_S sin(k theta) = k^2 sin(k theta)."""
    s = unit_circle()

    def u(Y):
        t = _theta(Y, s)
        return np.sin(t) + np.sin(12.0 * t)

    def f(Y):
        t = _theta(Y, s)
        return (1.0 + c) * np.sin(t) + (144.0 + c) * np.sin(12.0 * t)

    return Problem(s, c, f, u, "circle_sin12")


def sphere_l3(c: float = 1.0) -> Problem:
    """Unit sphere, u = (x^2 - y^2) z, a degree-3 harmonic polynomial (Re Y_3^2 up to scale)."""
    s = unit_sphere()

    def u(Y):
        d = _sphere_dirs(Y, s)
        return (d[:, 0] ** 2 - d[:, 1] ** 2) * d[:, 2]

    def f(Y):
        return (12.0 + c) * u(Y)

    return Problem(s, c, f, u, "sphere_l3")


def sphere_varcoef(c: float = 1.0) -> Problem:
    """Unit sphere, variable diffusion a = cos(phi) + 1.5 and u = cos(phi), phi the polar
    angle (cos(phi) = z): -div_S(a grad_S u) = 2 z (z + 1.5) - (1 - z^2)."""
    s = unit_sphere()

    def u(Y):
        return _sphere_dirs(Y, s)[:, 2]

    def a(Y):
        return u(Y) + 1.5

    def f(Y):
        z = u(Y)
        return 2.0 * z * (z + 1.5) - (1.0 - z * z) + c * z

    return Problem(s, c, f, u, "sphere_varcoef", a=a)


def dziuk_x1x2(c: float = 1.0) -> Problem:
    """Dziuk's level-set surface with u = x1 x2.  With n = grad(phi) / |grad(phi)| and
    kappa = div(n) = Lap(phi) / |grad(phi)| - grad(phi)^T Hess(phi) grad(phi) / |grad(phi)|^3,
    -Lap_S u = -Lap u + n^T Hess(u) n + kappa (n . grad u) = 2 n1 n2 + kappa (n1 x2 + n2 x1)."""
    s = dziuk_surface()

    def u(Y):
        X = Y - s.c0()
        return X[:, 0] * X[:, 1]

    def f(Y):
        X = Y - s.c0()
        x1, x2, x3 = X[:, 0], X[:, 1], X[:, 2]
        p = x1 - x3 * x3
        g = np.stack([2.0 * p, 2.0 * x2, 2.0 * x3 - 4.0 * x3 * p], axis=1)
        gn = np.sqrt(np.sum(g * g, axis=1))
        n = g / gn[:, None]
        h33 = 2.0 - 4.0 * p + 8.0 * x3 * x3
        lap = 4.0 + h33
        gHg = 2.0 * g[:, 0] ** 2 + 2.0 * g[:, 1] ** 2 + h33 * g[:, 2] ** 2 - 8.0 * x3 * g[:, 0] * g[:, 2]
        kappa = lap / gn - gHg / gn ** 3
        return 2.0 * n[:, 0] * n[:, 1] + kappa * (n[:, 0] * x2 + n[:, 1] * x1) + c * x1 * x2

    return Problem(s, c, f, u, "dziuk_x1x2")


def sphere_l5_paper(c: float = 1.0) -> Problem:
    """The paper's sphere harmonic cos(3 theta) sin^3(phi) (9 cos^2(phi) - 1), degree 5.

    -Lap_S u = 30 u, so f = (30 + c) u (the printed -29u is a misprint)."""
    s = unit_sphere()

    def u(Y):
        d = _sphere_dirs(Y, s)
        theta = np.arctan2(d[:, 1], d[:, 0])
        cphi = np.clip(d[:, 2], -1.0, 1.0)
        sphi = np.sqrt(np.maximum(0.0, 1.0 - cphi * cphi))
        return np.cos(3.0 * theta) * sphi ** 3 * (9.0 * cphi ** 2 - 1.0)

    def f(Y):
        return (30.0 + c) * u(Y)

    return Problem(s, c, f, u, "sphere_l5")


def torus_paper(R: float = 1.2, r: float = 0.6, c: float = 1.0) -> Problem:
    """Torus example of Sec. 4.6: u = sin(3 theta) + cos(2 phi) with its closed-form f."""
    s = torus(R, r)

    def u(Y):
        th, ph = _torus_angles(Y, s)
        return np.sin(3.0 * th) + np.cos(2.0 * ph)

    def f(Y):
        th, ph = _torus_angles(Y, s)
        rr = R + r * np.cos(ph)
        lap = (9.0 * np.sin(3.0 * th) / rr ** 2
               - 2.0 * np.sin(ph) * np.sin(2.0 * ph) / (r * rr)
               + 4.0 * np.cos(2.0 * ph) / r ** 2)
        return lap + c * (np.sin(3.0 * th) + np.cos(2.0 * ph))

    return Problem(s, c, f, u, "torus_paper")


def torus_modes(R: float, r: float, seed: int, c: float = 1.0) -> Problem:
    """Seeded mix of 16 torus Fourier modes a_mn cos(m theta + n phi + psi_mn),
    m = 1..4, n = 0..3, a ~ N(0,1), psi ~ U[0, 2 pi).  Every mode has m >= 1, so the
    mix integrates to zero over the torus (area element (R + r cos phi) r dtheta dphi).
    No closed-form solution (the modes are not Laplace-Beltrami eigenfunctions)."""
    s = torus(R, r)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((4, 4))
    psi = rng.uniform(0.0, 2.0 * math.pi, (4, 4))

    def f(Y):
        th, ph = _torus_angles(Y, s)
        out = np.zeros(Y.shape[0])
        for m in range(1, 5):
            for n in range(0, 4):
                out += a[m - 1, n] * np.cos(m * th + n * ph + psi[m - 1, n])
        return out

    return Problem(s, c, f, None, f"torus_modes_{seed}")


def _real_harmonic_basis(l: int, d: np.ndarray) -> List[np.ndarray]:
    """Real spherical harmonics of degree l at unit directions d (rows), via scipy."""
    from scipy.special import sph_harm_y

    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))  # polar
    phi = np.arctan2(d[:, 1], d[:, 0])  # azimuth
    out = []
    for m in range(0, l + 1):
        Y = sph_harm_y(l, m, theta, phi)
        out.append(np.real(Y))
        if m > 0:
            out.append(np.imag(Y))
    return out


def sphere_modes(R: float, seed: int, c: float = 1.0, center=(0.0, 0.0, 0.0)) -> Problem:
    """Seeded mix of real spherical harmonics of degree 1..4 with N(0,1) amplitudes.

    On a sphere of radius R a degree-l harmonic has -Lap_S Y = l(l+1)/R^2 Y, so the
    exact solution is sum a Y / (l(l+1)/R^2 + c)."""
    s = Surface(SPHERE, float(R), 0.0, tuple(center))
    rng = np.random.default_rng(seed)
    coefs = {l: rng.standard_normal(2 * l + 1) for l in range(1, 5)}

    def _parts(Y):
        d = (Y - s.c0()) / s.R
        return {l: _real_harmonic_basis(l, d) for l in coefs}

    def f(Y):
        P = _parts(Y)
        out = np.zeros(Y.shape[0])
        for l, a in coefs.items():
            for k, b in enumerate(P[l]):
                out += a[k] * b
        return out

    def u(Y):
        P = _parts(Y)
        out = np.zeros(Y.shape[0])
        for l, a in coefs.items():
            lam = l * (l + 1) / s.R ** 2 + c
            for k, b in enumerate(P[l]):
                out += a[k] * b / lam
        return out

    return Problem(s, c, f, u, f"sphere_modes_{seed}")


# ----------------------------------------------------------------------------
# solver configurations (grid spacing, levels, band radius, smoothing parameters)
# ----------------------------------------------------------------------------

LAM2_2D = 13.0  # band radius^2 / h^2 for bicubic stencils in 2-D
LAM2_3D = 17.0  # band radius^2 / h^2 for tricubic stencils in 3-D


@dataclass
class SolverConfig:
    name: str
    problem: Problem
    h0: float
    levels: int
    lam2: float
    nu1: int = 3
    nu2: int = 3
    omega: float = 2.0 / 3.0
    rtol: float = 1e-10
    max_cycles: int = 60


def config_circle(h_inv: int = 64, levels: int = 4) -> SolverConfig:
    """2-D FP64 workload: unit circle, h = 1/64 coarsened to 1/8, band radius sqrt(13) h."""
    return SolverConfig("circle_h%d" % h_inv, circle_sin12(), 1.0 / h_inv, levels, LAM2_2D)


def config_sphere(h_inv: int = 64, levels: int = 5) -> SolverConfig:
    """3-D FP64 workload: unit sphere, l = 3 harmonic, h = 1/64 coarsened to 1/4 (5 levels)."""
    return SolverConfig("sphere_h%d" % h_inv, sphere_l3(), 1.0 / h_inv, levels, LAM2_3D)


def config_sphere_varcoef(h_inv: int = 64, levels: int = 5) -> SolverConfig:
    """Variable-coefficient workload: unit sphere, a = z + 1.5, u = z, h = 1/64 to 1/4."""
    return SolverConfig("sphere_vc_h%d" % h_inv, sphere_varcoef(), 1.0 / h_inv, levels, LAM2_3D)


def config_dziuk(h_inv: int = 64, levels: int = 3) -> SolverConfig:
    """Level-set workload: Dziuk's surface, u = x1 x2, h = 1/64 coarsened to 1/16."""
    return SolverConfig("dziuk_h%d" % h_inv, dziuk_x1x2(), 1.0 / h_inv, levels, LAM2_3D)


def config_torus_mixed(h_inv: int = 256, levels: Optional[int] = None, seed_offset: int = 3) -> SolverConfig:
    """Mixed-precision workload: torus R = 1, r = 0.4, 16-mode RHS, coarsest h = 1/8."""
    if levels is None:
        levels = int(round(math.log2(h_inv / 8))) + 1
    return SolverConfig("torus_mixed_h%d" % h_inv, torus_modes(1.0, 0.4, SEED_BASE + seed_offset),
                        1.0 / h_inv, levels, LAM2_3D)


@dataclass
class BatchItem:
    problem: Problem
    h0: float
    levels: int
    lam2: float = LAM2_3D


def batch_problems(nprob: int = 256, seed: int = SEED_BASE + 4,
                   h_choices: Sequence[int] = (32, 64, 128), coarse_h_inv: int = 4) -> List[BatchItem]:
    """Uneven batch: half spheres R ~ U[0.5, 1.5], half tori R ~ U[0.8, 1.2], r ~ U[0.2, 0.5],
    h drawn uniformly from 1/32, 1/64, 1/128, random mode right-hand sides, each problem
    coarsened down to h = 1/coarse_h_inv (1/4 keeps every coarsest level below ~4.4k
    nodes, so the dense coarsest inverses of all problems fit together)."""
    rng = np.random.default_rng(seed)
    items = []
    for k in range(nprob):
        h_inv = int(rng.choice(np.asarray(h_choices)))
        levels = int(round(math.log2(h_inv / coarse_h_inv))) + 1
        sub = int(rng.integers(0, 2 ** 31 - 1))
        if k % 2 == 0:
            R = float(rng.uniform(0.5, 1.5))
            p = sphere_modes(R, sub)
        else:
            R = float(rng.uniform(0.8, 1.2))
            r = float(rng.uniform(0.2, 0.5))
            p = torus_modes(R, r, sub)
        items.append(BatchItem(p, 1.0 / h_inv, levels))
    return items


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded standard-normal vector (for operator parity checks)."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)
