"""Skeletonization (Sec. 5) through the C ABI against the FP64 reference
(oracle/skeleton.py): the ring ranks of the IDs, the lifted density of the
compressed solve against the full solution and against the reference's own
compressed solve, in FP64 and mixed precision; and a configuration too
tight for any proxy sphere, where the skeleton system is the full one.

Tolerances: ranks within 2 of the reference (the pivoted Gram-Schmidt and the
reference's Householder QR may order near-ties differently); densities within
1e-8 of the full solution at eps = 1e-8 and tol 1e-12 (the reference reaches
2.5e-10 on the two spheres)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(wl):
    from paper_1406_0236_amd import Context
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return ctx


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("which", ["two_spheres", "small"])
def test_skeleton_solve_matches_full_and_reference(which, c1_system, small_system):
    from oracle.multibody import gmres
    from oracle.skeleton import SkeletonSystem
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S = c1_system if which == "two_spheres" else small_system
    print(f"[gpu] skeleton {wl.name} N={wl.N}", flush=True)
    ctx = _ctx(wl)
    eps = 1e-8
    ns = ctx.skeletonize(eps, 2.0)
    K = SkeletonSystem(S, eps=eps, factor=2.0)
    for b, body in enumerate(S.bodies):
        k, ng = ctx.skeleton_rank(b)
        kr = K.ids[id(body.shape)][1].shape[1]
        print(f"body {b}: rings {k} of {ng} (reference {kr})")
        assert abs(k - kr) <= 2 and k <= ng
        if which == "two_spheres":
            assert k < 0.7 * ng
    assert abs(ns - K.Ns) <= 2 * max(b.shape.NF for b in S.bodies) * len(S.bodies)
    v = S.plane_waves(wl.dirs)[:, 0]
    x_full, _, _ = gmres(S.matvec, S.rhs(v), tol=1e-13)
    vd = ctx.incident_plane_waves(wl.dirs)
    for mode, tol in ((SOLVE_FP64, 1e-12), (SOLVE_MIXED, 1e-11)):
        sol, info = ctx.solve_skeleton(vd, mode=mode, tol=tol, max_iters=100, certify=True)
        x = sol.cpu().numpy()[0]
        e = _rel(x, x_full)
        print(f"mode {mode}: {info[0]['iterations']} iterations (inner {info[0]['inner_iterations']}), "
              f"full-system residual {info[0]['rel_residual']:.2e}, error vs full solution {e:.2e}")
        assert e < 1e-8, e
        assert info[0]["rel_residual"] < 1e-8
    # one GPU's share of the rows set: the compressed solve needs every row and refuses
    from paper_1406_0236_amd import AxsError
    ctx.set_target_bodies(1, 1)
    try:
        with pytest.raises(AxsError, match="target-body range"):
            ctx.solve_skeleton(vd, mode=SOLVE_MIXED, tol=1e-8, certify=True)
    finally:
        ctx.set_target_bodies(0, 0)
    xr, _ = K.solve(v, tol=1e-13)
    e = _rel(ctx.solve_skeleton(vd, mode=SOLVE_FP64, tol=1e-12)[0].cpu().numpy()[0], xr)
    print(f"vs the reference compressed solve: {e:.2e}")
    assert e < 1e-8
    ctx.close()


def test_skeleton_without_room_for_a_proxy_is_the_full_system():
    """Two unit spheres 0.3 apart: the largest proxy sphere that clears the
    neighbour (radius 1.3) lies so close to the body that the ID at 1e-8 keeps
    every ring, and the skeleton solve returns the full solution."""
    from paper_1406_0236_amd import SOLVE_FP64
    from workloads import configs
    wl = configs.two_spheres()
    wl.bodies[0].centre = np.array([-1.15, 0.0, 0.0])
    wl.bodies[1].centre = np.array([1.15, 0.0, 0.0])
    ctx = _ctx(wl)
    ns = ctx.skeletonize(1e-8, 2.0)
    assert ns == wl.N and ctx.skeleton_rank(0) == (100, 100)
    vd = ctx.incident_plane_waves(wl.dirs)
    full, _ = ctx.solve(vd, mode=SOLVE_FP64, tol=1e-12)
    sk, _ = ctx.solve_skeleton(vd, mode=SOLVE_FP64, tol=1e-12)
    e = float(torch.linalg.norm(sk - full) / torch.linalg.norm(full))
    print(f"no-proxy configuration: {e:.2e}")
    assert e < 1e-10
    ctx.close()


def test_skeleton_batched_solve_on_mixed_bodies():
    """The compressed system with 16 right-hand sides on the 8 mixed bodies
    (spheres, spheroids, bowls; kappa = 2 pi, discretised for 4 pi so that the
    rings are compressible): the skeleton context's batched
    inter-body sums (from 16 rhs the MFMA order with the FP16
    multiply-accumulate in FP32) inside the mixed solve; every lifted density
    within 5e-8 of the full FP64 solution and with a full-system residual
    below 5e-8 (the IDs at eps = 1e-8 leave 6e-9 here)."""
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    from workloads import configs
    wl = configs.mixed_bodies(n_dirs=16, disc_kappa=4 * np.pi)
    print(f"[gpu] skeleton batched {wl.name} N={wl.N}", flush=True)
    ctx = _ctx(wl)
    try:
        ns = ctx.skeletonize(1e-8, 2.0)
        print(f"skeleton unknowns {ns} of {wl.N}")
        assert ns < 0.8 * wl.N
        vd = ctx.incident_plane_waves(wl.dirs)
        full, info_f = ctx.solve(vd, mode=SOLVE_FP64, tol=1e-12, max_iters=200)
        assert all(i["converged"] for i in info_f)
        sol, info = ctx.solve_skeleton(vd, mode=SOLVE_MIXED, tol=1e-11, max_iters=100, certify=True)
        x, xf = sol.cpu().numpy(), full.cpu().numpy()
        errs = [_rel(x[c], xf[c]) for c in range(16)]
        res = [i["rel_residual"] for i in info]
        print(f"16 rhs: worst error vs full solution {max(errs):.2e}, worst full-system residual {max(res):.2e}, "
              f"inner iterations {info[0]['inner_iterations']}")
        assert max(errs) < 5e-8 and max(res) < 5e-8
    finally:
        ctx.close()
