"""Seeded synthetic geometry for rotationally symmetric scatterers.

This module only *generates inputs*: generating contours sampled at composite
Gauss-Legendre nodes (the tensor-product rule of Sec. 3.2, Remark "Convergence
order"), body poses, incident directions, interior point sources and exterior
targets.  It contains none of the method's arithmetic (no kernels, no modal
decomposition, no quadrature corrections, no solves); both the FP64 reference
implementation and the GPU library consume what it produces.

Conventions (shared by every consumer):
  * A contour is ``n_panels`` panels of ``p`` Gauss-Legendre nodes each,
    panel-major.  On each panel the local parameter is s in [-1, 1];
    ``rz[i] = (r, z)`` at the node and ``drz[i] = d(r, z)/ds`` there;
    ``gw[i]`` is the Gauss weight of the node on [-1, 1].
  * The contour runs from an axis point at the top to an axis point at the
    bottom, so the outward normal is (-z', r') / |gamma'| (Sec. 2, the
    combined-field jump relation with the +1/2 term requires the outward
    normal).
  * Body nodes are x = c + Rot (r cos th, r sin th, z) with th_l = 2 pi l / N_F.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def gauss_legendre(p: int):
    """p-point Gauss-Legendre nodes and weights on [-1, 1] (ascending)."""
    s, w = np.polynomial.legendre.leggauss(p)
    return s.astype(np.float64), w.astype(np.float64)


@dataclasses.dataclass
class Contour:
    """A generating curve sampled on a composite Gauss rule."""
    kind: str
    params: dict
    rz: np.ndarray      # (NG, 2) float64
    drz: np.ndarray     # (NG, 2) float64, derivative w.r.t. panel parameter s
    gw: np.ndarray      # (NG,) float64 Gauss weights on [-1, 1]
    n_panels: int
    p: int
    r_max: float        # max distance from the symmetry axis
    bound_radius: float  # radius of a ball about the body origin holding the body

    @property
    def NG(self) -> int:
        return self.rz.shape[0]


def _sample_pieces(pieces, p):
    """pieces: list of (f(t) -> (r, z, dr/dt, dz/dt), t0, t1, n_panels)."""
    s, w = gauss_legendre(p)
    rz, drz, gw = [], [], []
    npan = 0
    for f, t0, t1, n in pieces:
        edges = np.linspace(t0, t1, n + 1)
        for a, b in zip(edges[:-1], edges[1:]):
            t = 0.5 * (a + b) + 0.5 * (b - a) * s
            r, z, dr, dz = f(t)
            jac = 0.5 * (b - a)
            rz.append(np.stack([r, z], axis=1))
            drz.append(np.stack([dr * jac, dz * jac], axis=1))
            gw.append(w.copy())
            npan += 1
    return (np.concatenate(rz), np.concatenate(drz), np.concatenate(gw), npan)


def sphere(a: float, n_panels: int, p: int = 10) -> Contour:
    """Sphere of radius a: r = a sin t, z = a cos t, t from 0 (top) to pi."""
    f = lambda t: (a * np.sin(t), a * np.cos(t), a * np.cos(t), -a * np.sin(t))
    rz, drz, gw, npan = _sample_pieces([(f, 0.0, math.pi, n_panels)], p)
    return Contour("sphere", {"a": a}, rz, drz, gw, npan, p, a, a)


def prolate(a: float, c: float, n_panels: int, p: int = 10) -> Contour:
    """Spheroid with equatorial semi-axis a and polar semi-axis c (symmetry axis z)."""
    f = lambda t: (a * np.sin(t), c * np.cos(t), a * np.cos(t), -c * np.sin(t))
    rz, drz, gw, npan = _sample_pieces([(f, 0.0, math.pi, n_panels)], p)
    return Contour("prolate", {"a": a, "c": c}, rz, drz, gw, npan, p, a, max(a, c))


def bowl(n_inner: int, n_cap: int, n_outer: int, p: int = 10, R: float = 1.0,
         thick: float = 0.2, alpha_max: float = 2.0 * math.pi / 3.0) -> Contour:
    """Thick spherical-shell bowl (cavity opening upwards).

    Outer arc of radius R and inner arc of radius R - thick, both from the
    bottom pole (polar angle alpha = 0 measured from -z) to alpha_max, joined
    by a semicircular rim of radius thick/2.  The curve starts at the inner
    pole (the higher axis point), runs up the inner arc, over the rim and
    down the outer arc to the outer pole; it is C^1 at the junctions.
    """
    ri = R - thick
    rc = 0.5 * thick
    rm = R - rc
    ca, sa = math.cos(alpha_max), math.sin(alpha_max)
    # rim centre and the local radial / tangential unit vectors at alpha_max
    cen = np.array([rm * sa, -rm * ca])
    e_rho = np.array([sa, -ca])
    e_alp = np.array([ca, sa])

    def inner(t):
        return (ri * np.sin(t), -ri * np.cos(t), ri * np.cos(t), ri * np.sin(t))

    def cap(psi):
        r = cen[0] + rc * (-np.cos(psi) * e_rho[0] + np.sin(psi) * e_alp[0])
        z = cen[1] + rc * (-np.cos(psi) * e_rho[1] + np.sin(psi) * e_alp[1])
        dr = rc * (np.sin(psi) * e_rho[0] + np.cos(psi) * e_alp[0])
        dz = rc * (np.sin(psi) * e_rho[1] + np.cos(psi) * e_alp[1])
        return r, z, dr, dz

    def outer(u):  # u from 0 to alpha_max, alpha = alpha_max - u (descending)
        al = alpha_max - u
        return (R * np.sin(al), -R * np.cos(al), -R * np.cos(al), -R * np.sin(al))

    pieces = [(inner, 0.0, alpha_max, n_inner), (cap, 0.0, math.pi, n_cap),
              (outer, 0.0, alpha_max, n_outer)]
    rz, drz, gw, npan = _sample_pieces(pieces, p)
    r_max = float(np.max(rz[:, 0]))
    return Contour("bowl", {"R": R, "thick": thick, "alpha_max": alpha_max}, rz, drz, gw,
                   npan, p, max(R, r_max), R)


def panels_for_wavelength(length: float, kappa: float, min_panels: int = 1) -> int:
    """Panels of one piece at 10 nodes per wavelength (one panel per wavelength)."""
    lam = 2.0 * math.pi / kappa
    return max(min_panels, int(math.ceil(length / lam - 1e-12)))


def _prolate_length(a, c, n=20000):
    t = np.linspace(0, math.pi, n + 1)
    sp = np.hypot(a * np.cos(t), c * np.sin(t))
    return float(np.trapezoid(sp, t))


def sphere_at_wavelength(kappa, a=1.0, p=10):
    return sphere(a, panels_for_wavelength(math.pi * a, kappa), p)


def prolate_at_wavelength(kappa, a=1.0, c=2.0, p=10):
    return prolate(a, c, panels_for_wavelength(_prolate_length(a, c), kappa), p)


def bowl_at_wavelength(kappa, p=10, R=1.0, thick=0.2, alpha_max=2.0 * math.pi / 3.0):
    ri = R - thick
    n_in = panels_for_wavelength(ri * alpha_max, kappa)
    n_cap = panels_for_wavelength(math.pi * 0.5 * thick, kappa, min_panels=2)
    n_out = panels_for_wavelength(R * alpha_max, kappa)
    return bowl(n_in, n_cap, n_out, p, R, thick, alpha_max)


def modes_for(kappa: float, r_max: float, M_min: int = 20) -> int:
    """Fourier cutoff M = max(M_min, round(10 kappa r_max / pi))."""
    return max(M_min, int(round(10.0 * kappa * r_max / math.pi)))


# ----------------------------------------------------------------------------
# poses, directions, point sources
# ----------------------------------------------------------------------------

def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (unit quaternion from 4 normals)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def place_bodies(radii, box: float, gap: float, rng: np.random.Generator,
                 max_tries: int = 200000) -> np.ndarray:
    """Rejection-sample centres in [0, box]^3 so that bounding balls keep `gap`."""
    centres = []
    for rad in radii:
        for _ in range(max_tries):
            c = rng.uniform(rad, box - rad, size=3)
            if all(np.linalg.norm(c - c2) - rad - r2 >= gap for c2, r2 in centres):
                centres.append((c, rad))
                break
        else:
            raise RuntimeError("placement failed")
    return np.array([c for c, _ in centres])


def fibonacci_directions(n: int) -> np.ndarray:
    """n unit vectors on a Fibonacci sphere: z_i = 1 - (2i+1)/n, phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(n)
    z = 1.0 - (2.0 * i + 1.0) / n
    ph = i * math.pi * (3.0 - math.sqrt(5.0))
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(ph), rho * np.sin(ph), z], axis=1)


def uniform_directions(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def interior_point(contour: Contour, rng: np.random.Generator) -> np.ndarray:
    """A seeded point strictly inside the body (body frame)."""
    if contour.kind == "bowl":
        R, th = contour.params["R"], contour.params["thick"]
        rad = R - 0.5 * th
        alpha = math.radians(rng.uniform(20.0, 100.0))
        ph = rng.uniform(0, 2 * math.pi)
        return np.array([rad * math.sin(alpha) * math.cos(ph),
                         rad * math.sin(alpha) * math.sin(ph), -rad * math.cos(alpha)])
    if contour.kind == "sphere":
        inr = contour.params["a"]
    else:
        inr = min(contour.params["a"], contour.params["c"])
    v = rng.standard_normal(3)
    v /= np.linalg.norm(v)
    return v * rng.uniform(0.0, 0.5 * inr)


def uniform_interior_point(contour: Contour, rng: np.random.Generator) -> np.ndarray:
    """A seeded point uniformly distributed in the volume of a sphere or spheroid
    (body frame), by rejection from the bounding box."""
    if contour.kind not in ("sphere", "prolate"):
        raise ValueError("uniform interior points are defined for spheres and spheroids")
    a = contour.params["a"]
    c = contour.params.get("c", a)
    while True:
        x = rng.uniform(-1.0, 1.0, 3)
        if x @ x < 1.0:
            return x * np.array([a, a, c])


def sphere_targets(n: int, radius: float, centre, rng: np.random.Generator) -> np.ndarray:
    return np.asarray(centre) + radius * uniform_directions(n, rng)
