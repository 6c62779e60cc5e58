"""Parity tolerances derived from the arithmetic of each path.

FP32 inter-body sum (the ring and MFMA orders, and the point order): every
pair's phase kappa R / 2 pi is formed and rounded as an FP32 number of
revolutions from FP32 coordinates, an absolute phase error of about
kappa R 2^-24 radians, which is a relative error of the same size in the
pair's term; 1/sqrt, the hardware sin/cos, the products and the FP32
accumulation over the sources of one split add some tens of units in the
last place (40 seen at kappa = 0 with a single split of 3,060 sources).  With
random densities the errors of the terms add like their magnitudes, so the
sum's error relative to its largest entry is bounded by

    fp32_sum_bound = 2^-24 (kappa R_max + 64)

with R_max the largest distance between two nodes of the workload.  The FP16
multiply-accumulate keeps each product to 2^-20 (16 units of 2^-24), hence
`extra=16` for it.

Pairs much closer than the bodies' sizes: the ring and MFMA orders form R'^2
as |p|^2 - 2 y.p + |y|^2 in the source body's frame, whose rounding is
2^-24 (|p|^2 + |y|^2) against R'^2, i.e. a relative error of R of half of
2^-24 (|p|^2 + |y|^2) / R^2 (close_pair_bound).
"""
import math

import numpy as np

EPS32 = 2.0 ** -24


def rmax(wl):
    """Largest distance between two nodes: centre distance plus bounding radii."""
    c = np.array([b.centre for b in wl.bodies])
    r = np.array([b.contour.bound_radius for b in wl.bodies])
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=-1) + r[:, None] + r[None, :]
    return float(np.max(d)) if len(wl.bodies) > 1 else float(2 * r[0])


def fp32_sum_bound(wl, extra=0.0):
    return EPS32 * (wl.kappa * rmax(wl) + 64.0 + extra)


def close_pair_bound(wl):
    """Worst relative error of R from the |p|^2 - 2 y.p + |y|^2 form over body
    pairs: |p| <= centre distance + r_target, |y| <= r_source, R >= gap."""
    worst = 0.0
    for a, ba in enumerate(wl.bodies):
        for b, bb in enumerate(wl.bodies):
            if a == b:
                continue
            dist = float(np.linalg.norm(ba.centre - bb.centre))
            ra, rb = ba.contour.bound_radius, bb.contour.bound_radius
            gap = dist - ra - rb
            worst = max(worst, 0.5 * EPS32 * ((dist + ra) ** 2 + rb ** 2) / gap ** 2)
    return worst
