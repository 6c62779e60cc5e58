"""The paper's cavity observation (Sec. 6.2, Example 4): for bowl-shaped
cavities the block-diagonal preconditioner is essential -- without it GMRES
does not converge.  8 bowls 2 wavelengths across (kappa = 2 pi) with bounding
balls 0.5 apart, N = 110,160, one point source inside each wall; FP64 GMRES to
1e-9 through the C ABI.  (bench.py --cavities also runs 5 wavelengths.)"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_cavities_need_the_preconditioner():
    from paper_1406_0236_amd import SOLVE_FP64, Context
    from workloads import configs
    wl = configs.cavities_8()
    print(f"[gpu] {wl.name} N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    try:
        ctx.precompute_scattering()
        src = configs.point_sources(wl, seed=11)
        amp = np.random.default_rng(12).standard_normal(len(src))
        v = ctx.incident_point_sources(src, amp)
        sol, info = ctx.solve(v, mode=SOLVE_FP64, tol=1e-9, max_iters=150)
        xt = configs.exterior_targets(wl, 10, seed=12)
        d = np.linalg.norm(xt[:, None, :] - src[None, :, :], axis=-1)
        exact = -(np.exp(1j * wl.kappa * d) / (4.0 * math.pi * d)) @ amp
        u = ctx.eval_field(sol, xt).cpu().numpy()[0]
        err = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
        _, info_np = ctx.solve(v, mode=SOLVE_FP64, tol=1e-9, max_iters=150, precondition=False)
        print(f"preconditioned: {info[0]['iterations']} iterations, E_inf {err:.2e}; "
              f"without: {info_np[0]['iterations']} iterations, residual {info_np[0]['rel_residual']:.2e}")
        assert info[0]["converged"] and info[0]["iterations"] < 80
        assert err < 1e-3
        assert not info_np[0]["converged"] and info_np[0]["rel_residual"] > 1e-6
    finally:
        ctx.close()
