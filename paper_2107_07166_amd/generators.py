"""Seeded synthetic particle sets for the gravity solves.

This module only draws inputs: positions, masses and velocities of the
workloads the solver is exercised on.  It holds none of the force method's
arithmetic, so the CPU oracle and the GPU path can both be fed from it.

Every generator takes an explicit seed and uses numpy's PCG64 generator;
the workload seeds are 210707166 + the workload's index (see ``WORKLOADS``).

The workloads stand in for the paper's own test problems, which are not
reproducible from the text (the two "irregular shapes" of the distance test
and the white-dwarf SPH model are not specified numerically):

* uniform ball      -- equal masses, uniform in the unit sphere;
* Plummer sphere    -- scale radius a, equal masses, total mass 1;
* polytrope binary  -- two n=1 polytropes (density ~ sin(pi r)/(pi r)),
                       the gravity-only stand-in for the isolated star test;
* exponential disk  -- exponential surface density, sech^2 vertical profile.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 210707166


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors with an isotropic distribution (normalised Gaussians)."""
    v = rng.standard_normal((n, 3))
    nrm = np.sqrt((v * v).sum(axis=1))
    nrm[nrm == 0.0] = 1.0
    return v / nrm[:, None]


def uniform_ball(n: int, seed: int, radius: float = 1.0):
    """n equal masses (total 1) uniform in a ball: r = R U^(1/3)."""
    rng = _rng(seed)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    pos = _isotropic(rng, n) * r[:, None]
    mass = np.full(n, 1.0 / n)
    return np.ascontiguousarray(pos), mass


def plummer(n: int, seed: int, a: float = 1.0, u_max: float = 0.999,
            velocities: bool = False):
    """Plummer sphere of total mass 1 (G = 1).

    The enclosed-mass fraction u is drawn uniformly on [0, u_max) and the
    radius is r = a (u^(-2/3) - 1)^(-1/2); u_max = 0.999 truncates at about
    38.7 a.  Velocities (optional) use the Aarseth-Henon-Wielen rejection for
    q = v / v_esc with density q^2 (1 - q^2)^(7/2).
    """
    rng = _rng(seed)
    u = rng.random(n) * u_max
    u = np.maximum(u, 1e-300)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, n) * r[:, None]
    mass = np.full(n, 1.0 / n)
    if not velocities:
        return np.ascontiguousarray(pos), mass
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.random(todo.size)
        y = rng.random(todo.size) * 0.1
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0) * (1.0 + (r / a) ** 2) ** -0.25 / math.sqrt(a)
    vel = _isotropic(rng, n) * (q * vesc)[:, None]
    return np.ascontiguousarray(pos), mass, np.ascontiguousarray(vel)


def _polytrope_n1_radii(rng: np.random.Generator, n: int) -> np.ndarray:
    """Radii with enclosed-mass fraction (sin(pi r) - pi r cos(pi r)) / pi.

    This is the mass profile of a unit-radius n=1 polytrope, whose density is
    proportional to sin(pi r) / (pi r).  Inverted by 60 bisection steps.
    """
    u = rng.random(n)
    lo = np.zeros(n)
    hi = np.ones(n)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        f = (np.sin(math.pi * mid) - math.pi * mid * np.cos(math.pi * mid)) / math.pi
        below = f < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def polytrope_binary(n_each: int, seed: int, separation: float = 4.0,
                     star_mass: float = 0.5):
    """Two n=1 polytropes (radius 1) on a circular orbit, internally cold.

    Star centres at (-separation/2, 0, 0) and (+separation/2, 0, 0), bulk
    velocities (0, -v, 0) and (0, +v, 0) with v = sqrt(G M_tot / d) / 2.
    """
    rng = _rng(seed)
    pos = np.empty((2 * n_each, 3))
    vel = np.zeros((2 * n_each, 3))
    v_half = 0.5 * math.sqrt(2.0 * star_mass / separation)
    for s, sign in enumerate((-1.0, 1.0)):
        r = _polytrope_n1_radii(rng, n_each)
        p = _isotropic(rng, n_each) * r[:, None]
        p[:, 0] += sign * 0.5 * separation
        pos[s * n_each:(s + 1) * n_each] = p
        vel[s * n_each:(s + 1) * n_each, 1] = sign * v_half
    mass = np.full(2 * n_each, star_mass / n_each)
    return pos, mass, vel


def exponential_disk(n: int, seed: int, r_scale: float = 1.0, z_scale: float = 0.05,
                     r_max: float = 10.0, z_max: float = 0.5):
    """Exponential disk (total mass 1) with a sech^2 vertical profile.

    Cylindrical radius from 1 - (1 + R) e^(-R) = u (Newton), truncated at
    r_max scale lengths; z = z_scale * atanh(2u' - 1) clipped to |z| <= z_max;
    azimuth uniform.  Velocities are circular, v_c = sqrt(G M(<r) / r) with
    M(<r) counted from the sorted spherical radii.
    """
    rng = _rng(seed)
    u_cap = 1.0 - (1.0 + r_max) * math.exp(-r_max)
    u = rng.random(n) * u_cap
    R = np.where(u < 0.5, np.sqrt(2.0 * u) + 1e-12, 2.0)
    for _ in range(60):
        f = 1.0 - (1.0 + R) * np.exp(-R) - u
        df = R * np.exp(-R)
        R = np.clip(R - f / np.maximum(df, 1e-300), 1e-12, r_max)
    R = R * r_scale
    uz = rng.random(n)
    z = z_scale * np.arctanh(np.clip(2.0 * uz - 1.0, -1.0 + 1e-16, 1.0 - 1e-16))
    z = np.clip(z, -z_max, z_max)
    phi = rng.random(n) * (2.0 * math.pi)
    pos = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
    mass = np.full(n, 1.0 / n)
    rs = np.sqrt((pos * pos).sum(axis=1))
    order = np.argsort(rs, kind="stable")
    menc = np.empty(n)
    menc[order] = np.cumsum(mass[order])
    vc = np.sqrt(menc / np.maximum(rs, 1e-12))
    vel = np.stack([-vc * np.sin(phi), vc * np.cos(phi), np.zeros(n)], axis=1)
    return np.ascontiguousarray(pos), mass, np.ascontiguousarray(vel)


def _irregular_shape(rng: np.random.Generator, n: int) -> np.ndarray:
    """One irregular body: a union of 3-5 random ellipsoids (uniform density,
    rejection sampled), recentred on its centroid and scaled to unit maximum
    radius."""
    k = int(rng.integers(3, 6))
    centres = rng.normal(size=(k, 3)) * 0.45
    axes = rng.uniform(0.25, 0.7, size=(k, 3))
    rots = []
    for _ in range(k):
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        rots.append(q * np.sign(np.diag(r)))
    lo = (centres - axes.max(1, keepdims=True)).min(0)
    hi = (centres + axes.max(1, keepdims=True)).max(0)
    out = np.empty((0, 3))
    while len(out) < n:
        cand = lo + (hi - lo) * rng.random((4 * n, 3))
        inside = np.zeros(len(cand), dtype=bool)
        for c, a, q in zip(centres, axes, rots):
            u = (cand - c) @ q / a
            inside |= (u * u).sum(1) <= 1.0
        out = np.concatenate([out, cand[inside]])
    out = out[:n]
    out -= out.mean(0)
    return out / np.sqrt((out * out).sum(1)).max()


def irregular_pair(n_each: int, seed: int, separation: float):
    """Two irregular bodies of n_each particles (equal masses, total 1), unit
    maximum radius about their centres, with centres at -/+ (separation /
    (2 sqrt 3)) (1, 1, 1): distance `separation` along the cube diagonal, so
    for separation > 2 sqrt 3 each body sits in its own octant of the
    bounding cube."""
    rng = _rng(seed)
    c = separation / (2.0 * math.sqrt(3.0))
    a = _irregular_shape(rng, n_each) - c
    b = _irregular_shape(rng, n_each) + c
    return np.ascontiguousarray(np.concatenate([a, b])), np.full(2 * n_each, 0.5 / n_each)


@dataclass(frozen=True)
class Workload:
    """One named solve configuration: input recipe plus FMM parameters."""

    name: str
    index: int
    kind: str
    n: int
    p: int
    theta: float
    eps: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def seed(self) -> int:
        return SEED_BASE + self.index

    def make(self, n: int | None = None, velocities: bool = False):
        """Draw (pos, mass[, vel]) for this workload, optionally at another n."""
        n = self.n if n is None else int(n)
        if self.kind == "ball":
            pos, mass = uniform_ball(n, self.seed)
            vel = np.zeros_like(pos)
        elif self.kind == "plummer":
            pos, mass, vel = plummer(n, self.seed, velocities=True)
        elif self.kind == "binary":
            pos, mass, vel = polytrope_binary(n // 2, self.seed)
        elif self.kind == "disk":
            pos, mass, vel = exponential_disk(n, self.seed)
        else:
            raise ValueError(f"unknown workload kind {self.kind!r}")
        if velocities:
            return pos, mass, vel
        return pos, mass


WORKLOADS = {
    "ball2k": Workload("ball2k", 0, "ball", 2048, 2, 0.5),
    "plummer1m": Workload("plummer1m", 1, "plummer", 1 << 20, 4, 0.5),
    "binary4m": Workload("binary4m", 2, "binary", 1 << 22, 4, 0.7,
                         extra={"steps": 200, "dt": 1e-3}),
    "disk4m": Workload("disk4m", 3, "disk", 4194304, 6, 0.8),
}


def generate(kind: str, n: int, seed: int):
    """Draw (pos, mass) for one of the generator kinds at an explicit seed."""
    return Workload(kind, seed - SEED_BASE, kind, n, 1, 0.5).make()
