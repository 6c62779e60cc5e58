"""Properties of the exact scattering problem checked on the GPU solutions at
a realistic size, where the reference cannot solve: the 8 mixed bodies
(3 spheres, 3 spheroids, 2 bowl cavities; kappa = 2 pi, N = 16,810).

  * reciprocity of the far field, u_inf(x^; d) = u_inf(-d; -x^), for 4 x 4
    pairs of incident and observation directions;
  * the optical theorem, (4 pi / kappa) Im u_inf(d; d) = int_{S^2} |u_inf|^2,
    for 4 incident directions (Gauss-Legendre x trapezoid quadrature on the
    sphere of observation directions, through the library's far-field kernel).

Both hold for the exact solution; the discrete solution satisfies them to
its discretisation error (printed).  A sign or normalisation slip in the
operator, the solve or the far field breaks them by O(1)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_reciprocity_and_optical_theorem_on_mixed_bodies():
    from paper_1406_0236_amd import SOLVE_MIXED, Context
    from workloads import configs, geometry as geo
    wl = configs.mixed_bodies()
    print(f"[gpu] {wl.name} N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    try:
        ctx.precompute_scattering()
        rng = np.random.default_rng(17)
        d = geo.uniform_directions(4, rng)
        xh = geo.uniform_directions(4, rng)
        # incident d_i and -xh_j in one batched solve
        dirs = np.concatenate([d, -xh])
        v = ctx.incident_plane_waves(dirs)
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-11)
        assert all(i["converged"] for i in info)
        ff = ctx.far_field(sol, np.concatenate([xh, -d])).cpu().numpy()   # [8 rhs][8 directions]
        worst = 0.0
        for i in range(4):
            for j in range(4):
                a = ff[i, j]             # u_inf(xh_j; d_i)
                b = ff[4 + j, 4 + i]     # u_inf(-d_i; -xh_j)
                worst = max(worst, abs(a - b) / max(abs(a), abs(b)))
        print(f"reciprocity: worst relative difference {worst:.2e}")
        assert worst < 1e-5   # seen 1.5e-6
        nth, nph = 100, 200
        xg, wg = np.polynomial.legendre.leggauss(nth)
        ph = 2 * math.pi * np.arange(nph) / nph
        st = np.sqrt(1 - xg * xg)
        sph = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                        np.repeat(xg, nph)], axis=1)
        wq = np.repeat(wg, nph) * 2 * math.pi / nph
        uf = ctx.far_field(sol[:4].contiguous(), np.concatenate([sph, d])).cpu().numpy()
        worst_ot = 0.0
        for i in range(4):
            lhs = 4 * math.pi / wl.kappa * uf[i, sph.shape[0] + i].imag
            rhs = float(np.sum(wq * np.abs(uf[i, :sph.shape[0]]) ** 2))
            worst_ot = max(worst_ot, abs(lhs - rhs) / rhs)
        print(f"optical theorem: worst relative difference {worst_ot:.2e}")
        assert worst_ot < 1e-6   # seen 4.5e-8
    finally:
        ctx.close()
