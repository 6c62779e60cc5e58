"""Zero frequency (kappa = 0): the Laplace equation of Sec. 6.1, whose combined
field adds the single layer with the real coefficient eta (= 1), through the C
ABI against the FP64 reference on a sphere, a rotated spheroid and a rotated
bowl (tests/conftest.py::laplace_system).

Tolerances as in test_gpu_parity.py: modal matrices 2e-12 (3e-13 seen), FP64 sums
1e-13, FP32 sums fp32_sum_bound (2^-24 x 32 at kappa = 0), solves to 1e-11
within 1e-8 of the dense reference; the exterior
field of interior point sources within 1e-6 of the exact one (the reference
itself reaches 9e-9 on this discretisation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from tolerances import fp32_sum_bound  # noqa: E402


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.fixture(scope="module")
def lap(laplace_system):
    from paper_1406_0236_amd import Context
    wl, S = laplace_system
    print(f"[gpu] Laplace context {wl.name} N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return wl, S, ctx


def test_laplace_modal_matrices(lap):
    wl, S, ctx = lap
    for b, body in enumerate(S.bodies):
        sh = body.shape
        eA = rel(ctx.modal_matrices(b, 0, sh.M, sh.NG).cpu().numpy(), sh.modal_matrices())
        eS = rel(ctx.modal_matrices(b, 1, sh.M, sh.NG).cpu().numpy(), sh.inverses())
        print(f"body {b} ({wl.bodies[b].contour.kind}): A~ {eA:.2e} S {eS:.2e}")
        assert eA < 2e-12 and eS < 2e-12


def test_laplace_interbody_sum_all_orders(lap):
    """Point and ring orders (no phase: one rsq and a real kernel per pair), both
    precisions, several launch shapes; the MFMA order needs kappa > 0."""
    from paper_1406_0236_amd import FP32, FP64, AxsError
    wl, S, ctx = lap
    assert ctx.interbody_launch_shape(FP32)[0] == 2
    rng = np.random.default_rng(31)
    x = rng.standard_normal((5, S.N)) + 1j * rng.standard_normal((5, S.N))
    ref = S.apply_B(x.T).T
    for prec, tol in ((FP64, 1e-13), (FP32, fp32_sum_bound(wl))):
        for variant in (1, 2):
            for tpt, block, splits in ((1, 128, 1), (2, 256, 3), (4, 256, 0)):
                ctx.set_interbody_config(prec, variant, tpt, block, splits)
                e = rel(ctx.apply_interbody(_dev(x), prec).cpu().numpy(), ref)
                assert e < tol, (prec, variant, tpt, block, splits, e)
            print(f"prec {prec} variant {variant}: rel err {e:.2e}")
        ctx.set_interbody_config(prec, 3, 2, 256, 0)
        with pytest.raises(AxsError, match="EINVAL"):
            ctx.apply_interbody(_dev(x), prec)
        ctx.set_interbody_config(prec, 0, 0, 0, 0)


def test_laplace_solves_with_and_without_preconditioner(lap):
    """FP64 GMRES, mixed FGMRES and unpreconditioned FP64 GMRES on (D + B) sigma = -v
    all return the dense reference solution."""
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = lap
    from workloads import configs
    src = configs.point_sources(wl, seed=13)
    amp = np.array([1.0, -0.7, 0.0])
    v = S.point_source_field(src, amp, S.x)
    xd = S.solve_dense(v)
    vd = ctx.incident_point_sources(src, amp)
    assert rel(vd.cpu().numpy()[0], v) < 1e-13
    runs = ((SOLVE_FP64, True), (SOLVE_MIXED, True), (SOLVE_FP64, False))
    for mode, pre in runs:
        sol, info = ctx.solve(vd, mode=mode, tol=1e-11, max_iters=100, precondition=pre, certify=True)
        err = np.linalg.norm(sol.cpu().numpy()[0] - xd) / np.linalg.norm(xd)
        print(f"mode {mode} preconditioned {pre}: {info[0]['iterations']} iterations "
              f"(inner {info[0]['inner_iterations']}), residual {info[0]['rel_residual']:.1e}, err {err:.1e}")
        assert info[0]["converged"] and err < 1e-8, err
    # exterior field of the interior point sources (the accuracy protocol of Sec. 6)
    sol, _ = ctx.solve(vd, mode=SOLVE_MIXED, tol=1e-10)
    xt = configs.exterior_targets(wl, 10, seed=14)
    u = ctx.eval_field(sol, xt).cpu().numpy()[0]
    e = rel(u, -S.point_source_field(src, amp, xt))
    print(f"exterior field vs exact: {e:.2e}")
    assert e < 1e-6, e


def test_laplace_has_no_far_field(lap):
    from paper_1406_0236_amd import AxsError
    wl, S, ctx = lap
    x = torch.zeros((1, S.N), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(AxsError, match="EINVAL"):
        ctx.far_field(x, np.array([[0.0, 0.0, 1.0]]))


def test_laplace_125_spheroids_first_table_row():
    """The first row of the paper's 125-ellipsoid table (Sec. 6.1, fixture
    tests/golden/laplace_125_spheroids_table.txt): N_G = 50, N_F = 25, N =
    156,250 on the lattice reading of the geometry, FP64 GMRES to 1e-9.  The
    paper's observation at zero frequency -- the block-diagonal preconditioner
    makes no real difference (31 vs 33 iterations) -- must hold: the two
    iteration counts within 3 of each other and each within 5 of the printed
    one.  The field error depends on where the interior sources sit, which the
    paper does not state; with sources near the centres it is far below the
    printed 9.7e-5 and is only checked against 1e-6."""
    import math
    import os
    from paper_1406_0236_amd import SOLVE_FP64, Context
    from workloads import configs
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "laplace_125_spheroids_table.txt"))
    N, NG, NF, i_pre, i_no, e_paper = rows[0]
    wl = configs.laplace_ellipsoids(n_panels=int(NG) // 10, p=10, M=(int(NF) - 1) // 2)
    assert wl.N == int(N)
    print(f"[gpu] Laplace 125 spheroids N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    try:
        ctx.precompute_scattering()
        src = configs.point_sources(wl, seed=11)
        amp = np.random.default_rng(12).standard_normal(len(src))
        v = ctx.incident_point_sources(src, amp)
        its = {}
        for pre in (True, False):
            sol, info = ctx.solve(v, mode=SOLVE_FP64, tol=1e-9, precondition=pre)
            assert info[0]["converged"]
            its[pre] = info[0]["iterations"]
            if pre:
                xt = configs.exterior_targets(wl, 10, seed=12)
                u = ctx.eval_field(sol, xt).cpu().numpy()[0]
                d = xt[:, None, :] - src[None, :, :]
                exact = -(1.0 / (4.0 * math.pi * np.linalg.norm(d, axis=-1))) @ amp
                err = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
        print(f"iterations {its[True]} / {its[False]} (paper {int(i_pre)} / {int(i_no)}), "
              f"E_inf {err:.2e} (paper {e_paper:.2e})")
        assert abs(its[True] - its[False]) <= 3
        assert abs(its[True] - i_pre) <= 5 and abs(its[False] - i_no) <= 5
        assert err < 1e-6
    finally:
        ctx.close()
