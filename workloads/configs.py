"""The synthetic workloads (geometry, wavenumber, incident fields), seeded.

Every workload here is built from closed-form generating curves and seeded
numpy PCG64 streams; nothing is read from disk.  The paper's own experiments
(Sec. 6) do not publish their random placements, so these stand in for them
with the same kinds of bodies (spheres, prolate spheroids, bowl cavities),
sizes in wavelengths and separations.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

from . import geometry as geo


@dataclasses.dataclass
class BodySpec:
    contour: geo.Contour
    centre: np.ndarray   # (3,)
    rot: np.ndarray      # (3, 3)
    M: int               # Fourier cutoff; N_F = 2M + 1

    @property
    def n_nodes(self) -> int:
        return self.contour.NG * (2 * self.M + 1)


@dataclasses.dataclass
class Workload:
    name: str
    kappa: float
    eta: float
    bodies: list
    dirs: np.ndarray     # (nrhs, 3) plane-wave directions
    note: str = ""

    @property
    def N(self) -> int:
        return sum(b.n_nodes for b in self.bodies)

    @property
    def pairs(self) -> int:
        """Inter-body (target, source) pairs of one operator application."""
        n = np.array([b.n_nodes for b in self.bodies], dtype=np.int64)
        return int(n.sum() ** 2 - (n * n).sum())


def two_spheres(n_panels=10, p=10, M=20, kappa=math.pi) -> Workload:
    """Two unit spheres at (+-1.5, 0, 0), kappa = pi, eta = kappa, d = +z."""
    c = geo.sphere(1.0, n_panels, p)
    bodies = [BodySpec(c, np.array([s * 1.5, 0.0, 0.0]), np.eye(3), M) for s in (-1.0, 1.0)]
    return Workload("two_spheres_k1pi", kappa, kappa, bodies, np.array([[0.0, 0.0, 1.0]]),
                    "2 unit spheres, 10x10 Gauss nodes, |m|<=20, N=8200")


def sphere_lattice(n_panels=20, p=10, M=40, kappa=4 * math.pi, spacing=3.0, per_side=3) -> Workload:
    """27 unit spheres on a 3x3x3 lattice (spacing 3), kappa = 4 pi, d = (1,1,1)/sqrt3."""
    c = geo.sphere(1.0, n_panels, p)
    offs = (np.arange(per_side) - 0.5 * (per_side - 1)) * spacing
    bodies = [BodySpec(c, np.array(xyz, dtype=np.float64), np.eye(3), M)
              for xyz in itertools.product(offs, offs, offs)]
    d = np.ones((1, 3)) / math.sqrt(3.0)
    return Workload("sphere_lattice_27_k4pi", kappa, kappa, bodies, d,
                    "27 unit spheres 3x3x3 spacing 3, 20x10 Gauss nodes, |m|<=40, N=437400")


def mixed_bodies(seed=3, kappa=2 * math.pi, n_dirs=64, disc_kappa=None) -> Workload:
    """8 bodies in a 12^3 box, min gap 1: 3 spheres, 3 prolate 1x1x2, 2 bowls.

    ``disc_kappa`` sets the discretisation wavenumber (panels at 10 nodes per
    wavelength and the mode cutoff); it defaults to ``kappa``.
    """
    rng = np.random.default_rng(seed)
    kd = kappa if disc_kappa is None else disc_kappa
    shapes = ([geo.sphere_at_wavelength(kd)] * 3 + [geo.prolate_at_wavelength(kd)] * 3
              + [geo.bowl_at_wavelength(kd)] * 2)
    centres = geo.place_bodies([s.bound_radius for s in shapes], 12.0, 1.0, rng)
    bodies = []
    for s, c in zip(shapes, centres):
        rot = np.eye(3) if s.kind == "sphere" else geo.random_rotation(rng)
        bodies.append(BodySpec(s, c, rot, geo.modes_for(kd, s.r_max)))
    return Workload(f"mixed8_seed{seed}", kappa, kappa, bodies, geo.fibonacci_directions(n_dirs),
                    "3 spheres, 3 prolate 1x1x2, 2 bowls in 12^3, gap 1")


def mixed_many(seed=5, kappa=4 * math.pi, n_bodies=64, box=24.0, gap=0.5, n_dirs=16,
               p=10) -> Workload:
    """64 mixed bodies (spheres, spheroids of aspect U[1, 3], bowls) in a 24^3 box.

    Contours at the 27-sphere lattice's density (20 panels per pi of arc
    length, about 6.4 panels per wavelength at kappa = 4 pi), M from the
    equatorial radius.
    """
    rng = np.random.default_rng(seed)
    per_len = 20.0 / math.pi

    def npan(length, lo=1):
        return max(lo, int(math.ceil(length * per_len - 1e-9)))

    sph = geo.sphere(1.0, npan(math.pi), p)
    al = 2.0 * math.pi / 3.0
    bowl = geo.bowl(npan(0.8 * al), npan(0.1 * math.pi, 2), npan(al), p)
    shapes = []
    for b in range(n_bodies):
        kind = b % 3
        if kind == 0:
            shapes.append(sph)
        elif kind == 1:
            c = float(rng.uniform(1.0, 3.0))
            shapes.append(geo.prolate(1.0, c, npan(geo._prolate_length(1.0, c)), p))
        else:
            shapes.append(bowl)
    centres = geo.place_bodies([s.bound_radius for s in shapes], box, gap, rng)
    bodies = []
    for s, c in zip(shapes, centres):
        rot = np.eye(3) if s.kind == "sphere" else geo.random_rotation(rng)
        bodies.append(BodySpec(s, c, rot, geo.modes_for(kappa, s.r_max)))
    return Workload(f"mixed{n_bodies}_seed{seed}", kappa, kappa, bodies,
                    geo.fibonacci_directions(n_dirs), "64 mixed bodies in 24^3, gap 0.5")


def cavities_8(kappa=2 * math.pi, panels_per_unit=20.0 / math.pi, M=25, seed=4, p=10) -> Workload:
    """8 bowl cavities (outer radius 1, so 2 wavelengths across at kappa = 2 pi)
    on a 2 x 2 x 2 lattice whose bounding balls are 0.5 apart, each opening in a
    seeded uniform random direction; one point source inside each wall."""
    rng = np.random.default_rng(seed)

    def npan(length, lo=1):
        return max(lo, int(math.ceil(length * panels_per_unit - 1e-9)))

    al = 2.0 * math.pi / 3.0
    bw = geo.bowl(npan(0.8 * al), npan(0.1 * math.pi, 2), npan(al), p)
    step = 2.0 * bw.bound_radius + 0.5
    offs = bw.bound_radius + step * np.arange(2)
    bodies = [BodySpec(bw, np.array(xyz, dtype=np.float64), geo.random_rotation(rng), M)
              for xyz in itertools.product(offs, offs, offs)]
    return Workload(f"cavities8_k{kappa / math.pi:g}pi", kappa, kappa, bodies, np.array([[0.0, 0.0, 1.0]]),
                    "8 bowls, 2 x 2 x 2 lattice, bounding balls 0.5 apart, random orientations")


def laplace_small() -> Workload:
    """kappa = 0, eta = 1: unit sphere, spheroid 0.8 x 1.3 and a bowl, rotated, gaps > 0.5."""
    rng = np.random.default_rng(21)
    s = geo.sphere(1.0, 4, 10)
    pr = geo.prolate(0.8, 1.3, 5, 10)
    bw = geo.bowl(3, 2, 4, 10)
    bodies = [BodySpec(s, np.array([0.0, 0.0, 0.0]), np.eye(3), 8),
              BodySpec(pr, np.array([2.7, 0.4, -0.3]), geo.random_rotation(rng), 8),
              BodySpec(bw, np.array([-0.5, 2.6, 0.6]), geo.random_rotation(rng), 8)]
    return Workload("laplace_small", 0.0, 1.0, bodies, np.zeros((1, 3)),
                    "kappa = 0: sphere, spheroid, bowl")


def ellipsoids_8(kappa=10 * math.pi, n_panels=10, p=10, M=50) -> Workload:
    """8 prolate spheroids (axes 2 x 1 x 1, so 10 wavelengths long at kappa =
    10 pi) on a 2 x 2 x 2 lattice of spacing 2.05, long axes along z: the box
    is [0, 4.05] along z and neighbouring tips are 0.05 apart; eta = kappa."""
    c = geo.prolate(0.5, 1.0, n_panels, p)
    offs = 1.0 + 2.05 * np.arange(2)
    bodies = [BodySpec(c, np.array(xyz, dtype=np.float64), np.eye(3), M)
              for xyz in itertools.product(offs, offs, offs)]
    return Workload(f"ellipsoids8_k{kappa / math.pi:g}pi", kappa, kappa, bodies, np.array([[0.0, 0.0, 1.0]]),
                    "8 spheroids 2 x 1 x 1, 2^3 lattice, spacing 2.05")


def laplace_ellipsoids(per_side=5, spacing=2.05, n_panels=10, p=10, M=50, orient_seed=None) -> Workload:
    """125 prolate spheroids (axes 2 x 1 x 1) on a 5^3 lattice of spacing 2.05 inside
    [0, 10.2]^3; kappa = 0, eta = 1; 10 x 10 contour nodes x 101 azimuthal nodes =
    10,100 nodes per body.  By default all long axes lie along z, so neighbouring
    tips are 0.05 apart on their common axis; with orient_seed every body gets a
    seeded uniform random orientation (bounding balls stay 0.05 apart, so no two
    bodies come closer than 0.05, and close approaches are off the axes)."""
    c = geo.prolate(0.5, 1.0, n_panels, p)
    offs = 1.0 + spacing * np.arange(per_side)
    rng = np.random.default_rng(orient_seed) if orient_seed is not None else None
    bodies = [BodySpec(c, np.array(xyz, dtype=np.float64),
                       geo.random_rotation(rng) if rng is not None else np.eye(3), M)
              for xyz in itertools.product(offs, offs, offs)]
    tag = "" if orient_seed is None else f"_rot{orient_seed}"
    return Workload("laplace_ellipsoids_125" + tag, 0.0, 1.0, bodies, np.zeros((1, 3)),
                    "125 spheroids 2 x 1 x 1, 5^3 lattice, spacing 2.05, kappa = 0"
                    + ("" if orient_seed is None else ", random orientations"))


def single_sphere(a=1.0, n_panels=10, p=10, M=20, kappa=math.pi) -> Workload:
    c = geo.sphere(a, n_panels, p)
    return Workload("single_sphere", kappa, kappa, [BodySpec(c, np.zeros(3), np.eye(3), M)],
                    np.array([[0.0, 0.0, 1.0]]))


def point_sources(wl: Workload, seed: int = 11, uniform: bool = False):
    """One seeded point source strictly inside each body (global frame): within
    half the inradius of the centre (bowls: inside the wall), or with
    uniform=True uniformly distributed in the body's volume (spheres and
    spheroids)."""
    rng = np.random.default_rng(seed)
    pick = geo.uniform_interior_point if uniform else geo.interior_point
    return np.array([b.centre + b.rot @ pick(b.contour, rng) for b in wl.bodies])


def exterior_targets(wl: Workload, n: int = 10, seed: int = 12) -> np.ndarray:
    """n seeded targets on a sphere three wavelengths outside all bodies."""
    rng = np.random.default_rng(seed)
    cen = np.mean([b.centre for b in wl.bodies], axis=0)
    rad = max(np.linalg.norm(b.centre - cen) + b.contour.bound_radius for b in wl.bodies)
    lam = 2 * math.pi / wl.kappa if wl.kappa > 0 else 1.0
    return geo.sphere_targets(n, rad + 3 * lam, cen, rng)
