"""Parity of the HIP library (through the C ABI) with the FP64 reference.

Tolerances (relative to the largest entry of the compared quantity), each
within about 10x of what is seen and derived from the arithmetic where it is
not FP64 rounding (tests/tolerances.py):
  * setup matrices A~_m and S_m (FP64 on the device): MODAL_TOL = 2e-12 -- both
    sides integrate the same exact integrals, the reference to its rounding
    floor (5e-13), the device with a graded Gauss rule; 9e-14 to 3e-13 seen on
    spheres and the small spheroid.  COARSE_SPHEROID_TOL = 5e-11 where a
    spheroid has 5 or fewer panels: on the near panels of its pole-adjacent
    targets (r ~ 0.01) the two rules differ by up to 2.5e-11 (both converged
    under their own refinement; far entries agree to 4e-16);
  * FP64 inter-body sum: FP64_TOL = 1e-13 (2e-15 to 3e-14 seen); with the
    per-mode inverses in it (preconditioner, operator): FP64_OP_TOL = 1e-12
    (1.2e-13 seen: the inverses' agreement);
  * FP32 inter-body sum and operator: fp32_sum_bound = 2^-24 (kappa R_max + 64)
    -- each pair's phase rounded as FP32 revolutions (kappa R 2^-24) plus the
    rounding of 1/sqrt, the hardware sin/cos and the sums; 2^-20 more per
    product for the FP16 multiply-accumulate; pairs far closer than the
    bodies' sizes add the cancellation of |p|^2 - 2 y.p + |y|^2
    (close_pair_bound);
  * solves to tol 1e-11: 1e-8 (condition number of the second-kind system times tol).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tolerances import close_pair_bound, fp32_sum_bound  # noqa: E402

MODAL_TOL = 2e-12
COARSE_SPHEROID_TOL = 5e-11
FP64_TOL = 1e-13
FP64_OP_TOL = 1e-12


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _ctx_for(wl):
    from paper_1406_0236_amd import Context
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return ctx


@pytest.fixture(scope="module")
def small(small_system):
    wl, S = small_system
    print(f"[gpu] building context for {wl.name} N={wl.N}", flush=True)
    return wl, S, _ctx_for(wl)


def _rand(n, r, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


# --------------------------------------------------------------------------
# setup: modal matrices and their inverses
# --------------------------------------------------------------------------

def test_modal_matrices_match_reference(small):
    wl, S, ctx = small
    for bid, body in enumerate(S.bodies):
        sh = body.shape
        A_gpu = ctx.modal_matrices(bid, 0, sh.M, sh.NG).cpu().numpy()
        S_gpu = ctx.modal_matrices(bid, 1, sh.M, sh.NG).cpu().numpy()
        e_a = rel(A_gpu, sh.modal_matrices())
        e_s = rel(S_gpu, sh.inverses())
        print(f"body {bid}: A~ rel err {e_a:.2e}, S rel err {e_s:.2e}")
        assert e_a < MODAL_TOL and e_s < MODAL_TOL


def test_node_geometry_matches_reference(small):
    wl, S, ctx = small
    g = ctx.node_geometry()
    assert rel(g[:, :3], S.x) < 1e-14
    assert rel(g[:, 3:6], S.n) < 1e-14
    assert rel(g[:, 6], S.w) < 1e-14


# --------------------------------------------------------------------------
# operator pieces
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_interbody_sum_fp64_and_fp32(small, nrhs):
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    sig = _rand(S.N, nrhs, 10 + nrhs)
    ref = S.apply_B(sig.T).T
    y64 = ctx.apply_interbody(_dev(sig), FP64).cpu().numpy()
    y32 = ctx.apply_interbody(_dev(sig), FP32).cpu().numpy()
    assert rel(y64, ref) < FP64_TOL, rel(y64, ref)
    assert rel(y32, ref) < fp32_sum_bound(wl), rel(y32, ref)


def test_preconditioner_matches_reference(small):
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    x = _rand(S.N, 2, 21)
    ref = S.apply_Dinv(x.T).T
    y64 = ctx.apply_precond(_dev(x), FP64).cpu().numpy()
    y32 = ctx.apply_precond(_dev(x), FP32).cpu().numpy()
    print(f"preconditioner: FP64 {rel(y64, ref):.2e}, FP32 {rel(y32, ref):.2e}")
    assert rel(y64, ref) < FP64_OP_TOL, rel(y64, ref)
    assert rel(y32, ref) < fp32_sum_bound(wl), rel(y32, ref)


@pytest.mark.parametrize("nrhs", [1, 4])
def test_preconditioned_operator(small, nrhs):
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    sig = _rand(S.N, nrhs, 30 + nrhs)
    ref = np.stack([S.matvec(s) for s in sig])
    y64 = ctx.apply_matvec(_dev(sig), FP64).cpu().numpy()
    y32 = ctx.apply_matvec(_dev(sig), FP32).cpu().numpy()
    print(f"operator, {nrhs} rhs: FP64 {rel(y64, ref):.2e}, FP32 {rel(y32, ref):.2e}")
    assert rel(y64, ref) < FP64_OP_TOL, rel(y64, ref)
    assert rel(y32, ref) < fp32_sum_bound(wl), rel(y32, ref)


def test_operator_is_bitwise_reproducible(small):
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    x = _dev(_rand(S.N, 2, 41))
    for prec in (FP64, FP32):
        a = ctx.apply_matvec(x, prec).cpu().numpy()
        b = ctx.apply_matvec(x, prec).cpu().numpy()
        assert np.array_equal(a, b)


def test_interbody_launch_shapes_agree(small):
    """Every launch shape and source order computes the same sum (tiles, splits, ragged tails)."""
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    x = _dev(_rand(S.N, 3, 43))
    ref = S.apply_B(x.cpu().numpy().T).T
    for prec, tol in ((FP64, FP64_TOL), (FP32, fp32_sum_bound(wl))):
        for variant in (1, 2):
            for tpt, block, splits in ((1, 128, 1), (2, 256, 3), (4, 256, 7), (8, 256, 2), (4, 128, 16)):
                ctx.set_interbody_config(prec, variant, tpt, block, splits)
                y = ctx.apply_interbody(x, prec).cpu().numpy()
                e = rel(y, ref)
                assert e < tol, (prec, variant, tpt, block, splits, e)
            print(f"prec {prec} variant {variant}: last rel err {e:.2e}")
        ctx.set_interbody_config(prec, 0, 0, 0, 0)


@pytest.mark.parametrize("M, fits128", [(127, True), (128, False)])
def test_ring_order_at_the_tile_limit(M, fits128):
    """A ring of N_F = 2M + 1 azimuths is staged as N_F/2 + 1 mirror-pair entries
    (azimuth 0 alone, then l with N_F - l); 128-thread blocks hold rings of up to
    128 entries (M = 127) and refuse wider ones, 256-thread blocks take both."""
    from oracle.multibody import System
    from paper_1406_0236_amd import FP32, FP64, AxsError, Context
    from workloads import configs
    wl = configs.two_spheres(n_panels=2, p=4, M=M)
    S = System.from_workload(wl)
    print(f"[gpu] ring tile limit M={M} N={S.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    x = _dev(_rand(S.N, 2, 47))
    ref = S.apply_B(x.cpu().numpy().T).T
    for prec, tol in ((FP64, FP64_TOL), (FP32, fp32_sum_bound(wl))):
        for block in (128, 256):
            ctx.set_interbody_config(prec, 2, 1, block, 0)
            if block == 128 and not fits128:
                with pytest.raises(AxsError, match="EINVAL"):
                    ctx.apply_interbody(x, prec)
                continue
            e = rel(ctx.apply_interbody(x, prec).cpu().numpy(), ref)
            print(f"prec {prec} block {block}: rel err {e:.2e}")
            assert e < tol, (prec, block, e)
    ctx.close()


def test_fp64_interbody_is_accurate_to_rounding(small):
    """The FP64 sum (own octant-reduced sin/cos, Newton-refined 1/sqrt) agrees with
    the reference to a few ulps of the largest term, for both source orders."""
    from paper_1406_0236_amd import FP64
    wl, S, ctx = small
    sig = _rand(S.N, 1, 44)
    ref = S.apply_B(sig.T).T
    for variant in (1, 2):
        ctx.set_interbody_config(FP64, variant, 0, 0, 0)
        y = ctx.apply_interbody(_dev(sig), FP64).cpu().numpy()
        e = rel(y, ref)
        print(f"variant {variant}: FP64 rel err {e:.2e}")
        assert e < 1e-13, e
    ctx.set_interbody_config(FP64, 0, 0, 0, 0)


# --------------------------------------------------------------------------
# incident fields, field evaluation
# --------------------------------------------------------------------------

def test_incident_fields_and_field_evaluation(small):
    wl, S, ctx = small
    dirs = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]])
    v = ctx.incident_plane_waves(dirs).cpu().numpy()
    assert rel(v, S.plane_waves(dirs).T) < 1e-13
    src = np.array([[0.1, 0.2, -0.1], [2.5, 0.5, -0.2]])
    amp = np.array([1.0 + 0.5j, -0.3j])
    vp = ctx.incident_point_sources(src, amp).cpu().numpy()[0]
    assert rel(vp, S.point_source_field(src, amp, S.x)) < 1e-13
    sig = _rand(S.N, 2, 51)
    tg = np.array([[5.0, 1.0, 2.0], [-4.0, 3.0, 0.5], [0.5, 0.5, 6.0]])
    u = ctx.eval_field(_dev(sig), tg).cpu().numpy()
    assert rel(u, S.eval_field(sig.T, tg).T) < 1e-12
    xh = np.array([[0.0, 0.0, 1.0], [0.6, 0.8, 0.0]])
    uf = ctx.far_field(_dev(sig), xh).cpu().numpy()
    assert rel(uf, S.far_field(sig.T, xh).T) < 1e-12


# --------------------------------------------------------------------------
# solves
# --------------------------------------------------------------------------

def test_solves_match_dense_reference(small):
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = small
    dirs = np.array([[0.0, 0.6, 0.8], [0.48, -0.6, 0.64]])
    v = S.plane_waves(dirs)
    xd = np.stack([S.solve_dense(v[:, c]) for c in range(2)])
    vd = ctx.incident_plane_waves(dirs)
    for mode in (SOLVE_FP64, SOLVE_MIXED):
        sol, info = ctx.solve(vd, mode=mode, tol=1e-11, max_iters=100)
        x = sol.cpu().numpy()
        err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
        print(f"mode {mode}: {info} err {err:.2e}")
        assert err < 1e-8, err
        assert all(i["converged"] for i in info)
        assert all(i["rel_residual"] <= 1e-11 for i in info)


def test_gmres_residual_equals_explicit_residual(small):
    """The residual GMRES reports (least squares in its FP64 Arnoldi basis) is the
    explicit FP64 residual of the returned sigma up to rounding: the certified
    solve (one more FP64 application) returns the same sigma bit for bit and a
    residual within 1e-13 of it, for both solvers."""
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = small
    vd = ctx.incident_plane_waves(np.array([[0.0, 0.6, 0.8], [0.48, -0.6, 0.64]]))
    for mode in (SOLVE_FP64, SOLVE_MIXED):
        x1, i1 = ctx.solve(vd, mode=mode, tol=1e-9, max_iters=100)
        x2, i2 = ctx.solve(vd, mode=mode, tol=1e-9, max_iters=100, certify=True)
        assert torch.equal(x1, x2)
        for a, b in zip(i1, i2):
            print(f"mode {mode}: GMRES {a['rel_residual']:.3e} explicit {b['rel_residual']:.3e}")
            assert abs(a["rel_residual"] - b["rel_residual"]) <= 1e-13
            assert a["converged"] and b["converged"]


def test_augmented_inner_runs_against_restarted_ones(small, mixed):
    """Mixed solves whose later inner GMRES runs are augmented with the first
    inner run's Krylov space (the default) against inner runs restarted from
    scratch (AXS_SOLVE_RESTART_INNER), to tol 1e-11 (several outer steps, so
    several augmented runs): both certified by the explicit FP64 residual,
    both within 1e-8 of the dense reference solve (two bodies, 3 directions)
    and of each other (8 bodies, 64 directions, tol 1e-9), and the augmented
    runs never take more inner iterations.  The flag is refused in FP64 mode."""
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED, SOLVE_RESTART_INNER, AxsError
    wl, S, ctx = small
    dirs = np.array([[0.0, 0.6, 0.8], [0.48, -0.6, 0.64], [-0.8, 0.0, 0.6]])
    v = S.plane_waves(dirs)
    xd = np.stack([S.solve_dense(v[:, c]) for c in range(3)])
    vd = ctx.incident_plane_waves(dirs)
    inner = {}
    for name, mode in (("augmented", SOLVE_MIXED), ("restarted", SOLVE_MIXED | SOLVE_RESTART_INNER)):
        sol, info = ctx.solve(vd, mode=mode, tol=1e-11, max_iters=100, certify=True)
        err = np.linalg.norm(sol.cpu().numpy() - xd) / np.linalg.norm(xd)
        inner[name] = sum(i["inner_iterations"] for i in info)
        print(f"{name}: outer {[i['iterations'] for i in info]} inner {inner[name]} err {err:.2e}")
        assert all(i["converged"] and i["rel_residual"] <= 1e-11 for i in info)
        assert err < 1e-8, err
    assert inner["augmented"] <= inner["restarted"]
    with pytest.raises(AxsError, match="EINVAL"):
        ctx.solve(vd, mode=SOLVE_FP64 | SOLVE_RESTART_INNER, tol=1e-9)

    wl, S, ctx = mixed
    vd = ctx.incident_plane_waves(wl.dirs)
    sols, inner = [], {}
    for name, mode in (("augmented", SOLVE_MIXED), ("restarted", SOLVE_MIXED | SOLVE_RESTART_INNER)):
        sol, info = ctx.solve(vd, mode=mode, tol=1e-9, max_iters=100, certify=True)
        inner[name] = sum(i["inner_iterations"] for i in info)
        print(f"{name}: inner iterations over 64 rhs {inner[name]}")
        assert all(i["converged"] and i["rel_residual"] <= 1e-9 for i in info)
        sols.append(sol.cpu().numpy())
    d = np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1])
    print(f"augmented vs restarted: {d:.2e}")
    assert d < 1e-7, d
    assert inner["augmented"] <= inner["restarted"]


def test_mixed_solve_with_a_zero_incident_field(small):
    """A batch whose middle incident field is zero: its first inner run breaks
    down at once (a zero Arnoldi vector), so it is left out of the augmentation
    of the later inner runs while the other two keep it.  The zero column
    comes back exactly zero and converged, the others match the dense
    reference solve, for the augmented and the restarted inner runs alike."""
    from paper_1406_0236_amd import SOLVE_MIXED, SOLVE_RESTART_INNER
    wl, S, ctx = small
    dirs = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0], [-0.8, 0.0, 0.6]])
    v = S.plane_waves(dirs)
    vd = ctx.incident_plane_waves(dirs)
    vd[1].zero_()
    xd = [S.solve_dense(v[:, c]) for c in (0, 2)]
    for mode in (SOLVE_MIXED, SOLVE_MIXED | SOLVE_RESTART_INNER):
        sol, info = ctx.solve(vd, mode=mode, tol=1e-10, max_iters=100, certify=True)
        x = sol.cpu().numpy()
        print(mode, [(i["iterations"], i["inner_iterations"], i["rel_residual"]) for i in info])
        assert np.all(x[1] == 0) and info[1]["converged"]
        for c, ref in zip((0, 2), xd):
            err = np.linalg.norm(x[c] - ref) / np.linalg.norm(ref)
            assert info[c]["converged"] and err < 1e-8, (mode, c, err)


def test_warm_start_is_used_and_bad_guess_is_dropped(small):
    from paper_1406_0236_amd import SOLVE_FP64
    wl, S, ctx = small
    vd = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve(vd, mode=SOLVE_FP64, tol=1e-10)
    # exact guess: kept, converges immediately
    sol2, info2 = ctx.solve(vd, sigma0=sol.clone(), mode=SOLVE_FP64, tol=1e-9)
    assert info2[0]["used_warm_start"] == 1 and info2[0]["iterations"] == 0
    # absurd guess: residual above ||b||, replaced by zero
    bad = sol * 1e3
    sol3, info3 = ctx.solve(vd, sigma0=bad, mode=SOLVE_FP64, tol=1e-10)
    assert info3[0]["used_warm_start"] == 0
    assert np.linalg.norm((sol3 - sol).cpu().numpy()) <= 1e-8 * np.linalg.norm(sol.cpu().numpy())


def test_mixed_solve_takes_the_guess_into_its_first_preconditioner_step(small):
    """Mixed mode: a good guess enters the first flexible-preconditioner step
    (kept, fewer FP32 iterations, the same FP64-certified answer); a guess whose
    FP32 residual exceeds ||b|| is dropped and the solve is bit for bit the one
    from zero."""
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = small
    vd = ctx.incident_plane_waves(wl.dirs)
    sol, _ = ctx.solve(vd, mode=SOLVE_FP64, tol=1e-12)
    zero, iz = ctx.solve(vd, mode=SOLVE_MIXED, tol=1e-9, certify=True)
    warm, iw = ctx.solve(vd, sigma0=(sol * (1 + 1e-3)).contiguous(), mode=SOLVE_MIXED, tol=1e-9, certify=True)
    print(f"mixed from zero: {iz[0]}; from the guess: {iw[0]}")
    assert iw[0]["used_warm_start"] == 1 and iw[0]["converged"] and iw[0]["rel_residual"] <= 1e-9
    assert iw[0]["inner_iterations"] < iz[0]["inner_iterations"]
    assert np.linalg.norm((warm - sol).cpu().numpy()) <= 1e-7 * np.linalg.norm(sol.cpu().numpy())
    bad, ib = ctx.solve(vd, sigma0=sol * 1e3, mode=SOLVE_MIXED, tol=1e-9, certify=True)
    assert ib[0]["used_warm_start"] == 0
    assert torch.equal(bad, zero)


def test_not_converged_status(small):
    from paper_1406_0236_amd import SOLVE_FP64
    wl, S, ctx = small
    vd = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve(vd, mode=SOLVE_FP64, tol=1e-12, max_iters=1)
    assert info[0]["converged"] == 0 and info[0]["iterations"] == 1


# --------------------------------------------------------------------------
# error paths through the ABI
# --------------------------------------------------------------------------

def test_error_paths():
    from paper_1406_0236_amd import AxsError, Context, FP64
    from workloads import geometry as geo
    s = geo.sphere(1.0, 3, 10)
    ctx = Context(0)
    x = torch.zeros((1, 1), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(AxsError, match="ESTATE"):
        ctx.precompute_scattering()
    ctx.build_body(s.rz, s.drz, s.gw, s.n_panels, s.p, 1.0, 1.0, 4, [0, 0, 0], np.eye(3))
    with pytest.raises(AxsError, match="EINVAL"):   # overlapping bodies
        ctx.build_body(s.rz, s.drz, s.gw, s.n_panels, s.p, 1.0, 1.0, 4, [1.0, 0, 0], np.eye(3))
    with pytest.raises(AxsError, match="EINVAL"):   # kappa mismatch
        ctx.build_body(s.rz, s.drz, s.gw, s.n_panels, s.p, 2.0, 2.0, 4, [5.0, 0, 0], np.eye(3))
    with pytest.raises(AxsError, match="EINVAL"):   # wrong Gauss weights
        ctx.build_body(s.rz, s.drz, s.gw * 1.01, s.n_panels, s.p, 1.0, 1.0, 4, [5.0, 0, 0], np.eye(3))
    bad = s.rz.copy()
    bad[3, 0] = np.nan
    with pytest.raises(AxsError, match="ENONFINITE"):
        ctx.build_body(bad, s.drz, s.gw, s.n_panels, s.p, 1.0, 1.0, 4, [5.0, 0, 0], np.eye(3))
    with pytest.raises(AxsError, match="EINVAL"):   # rotation not orthonormal
        ctx.build_body(s.rz, s.drz, s.gw, s.n_panels, s.p, 1.0, 1.0, 4, [5.0, 0, 0], 2 * np.eye(3))
    y = torch.zeros((1, ctx.N), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(AxsError, match="ESTATE"):   # matvec before precompute
        ctx.apply_matvec(y.clone(), FP64, out=y)
    ctx.precompute_scattering()
    with pytest.raises(AxsError, match="ESTATE"):   # no bodies after precompute
        ctx.build_body(s.rz, s.drz, s.gw, s.n_panels, s.p, 1.0, 1.0, 4, [5.0, 0, 0], np.eye(3))
    with pytest.raises(AxsError, match="EINVAL"):   # output overlaps input
        ctx.apply_matvec(y, FP64, out=y)
    empty = torch.zeros((0, ctx.N), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(AxsError, match="EINVAL"):   # no right-hand sides
        ctx.apply_matvec(empty, FP64)
    with pytest.raises(AxsError, match="EINVAL"):
        ctx.solve(empty)
    with pytest.raises(AxsError, match="EINVAL"):   # no such source order
        ctx.set_interbody_config(FP64, 5, 2, 256, 0)
    # a single body: no inter-body terms, the operator is the identity
    z = torch.from_numpy(_rand(ctx.N, 1, 3)).to("cuda:0")
    assert torch.equal(ctx.apply_matvec(z, FP64), z)
    ctx.close()


# --------------------------------------------------------------------------
# the two-sphere workload (kappa = pi, N = 8200)
# --------------------------------------------------------------------------

def test_nonfinite_inputs_are_refused(small):
    """A NaN or Inf in the incident field stops the solve with AXS_ENONFINITE; a NaN
    or Inf density stops axs_apply_matvec, axs_apply_interbody and
    axs_apply_precond before anything is computed (the output is left as it
    was); a non-finite initial guess is not kept (the zero guess is used) and
    the solve converges."""
    from paper_1406_0236_amd import AxsError, FP32, FP64, SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = small
    v = ctx.incident_plane_waves(wl.dirs)
    for bad in (float("nan"), float("inf")):
        vb = v.clone()
        vb[0, S.N // 2] = complex(bad, 0.0)
        for mode in (SOLVE_FP64, SOLVE_MIXED):
            with pytest.raises(AxsError, match="ENONFINITE"):
                ctx.solve(vb, mode=mode, tol=1e-8)
        x = _dev(_rand(S.N, 2, 31))
        x[1, 7] = complex(0.0, bad)
        for fn in (ctx.apply_matvec, ctx.apply_interbody, ctx.apply_precond):
            for prec in (FP64, FP32):
                out = torch.full_like(x, 3.0)
                with pytest.raises(AxsError, match="ENONFINITE"):
                    fn(x, prec, out=out)
                assert torch.all(out == 3.0)
    guess = torch.full_like(v, float("nan"))
    sol, info = ctx.solve(v, sigma0=guess, mode=SOLVE_MIXED, tol=1e-9)
    assert info[0]["used_warm_start"] == 0 and info[0]["converged"]
    ref, _ = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-9)
    assert torch.equal(sol, ref)


@pytest.fixture(scope="module")
def c1(c1_system):
    wl, S = c1_system
    print(f"[gpu] building context for {wl.name} N={wl.N}", flush=True)
    return wl, S, _ctx_for(wl)


def test_two_spheres_modal_matrices(c1):
    wl, S, ctx = c1
    sh = S.bodies[0].shape
    e = rel(ctx.modal_matrices(0, 1, sh.M, sh.NG).cpu().numpy(), sh.inverses())
    print("S rel err", e)
    assert e < MODAL_TOL


def test_two_spheres_operator_fp32_and_fp64(c1):
    """The benchmark's small case (two spheres, kappa = pi, N = 8,200): the whole
    preconditioned operator in both precisions against the reference on two
    random densities.  FP32 within 1e-6 (the FP32 phase error kappa R 2^-24 is
    9e-7 at R_max = 5; the FP32 part is D^{-1} B sigma, about a third of the
    largest entry), FP64 within 1e-12."""
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = c1
    sig = _rand(S.N, 2, 101)
    ref = np.stack([S.matvec(c) for c in sig])
    for prec, tol in ((FP64, FP64_OP_TOL), (FP32, 1e-6)):
        e = rel(ctx.apply_matvec(_dev(sig), prec).cpu().numpy(), ref)
        print(f"two spheres, precision {prec}: operator rel err {e:.2e} (bound {tol:.1e})")
        assert e < tol, e


def test_two_spheres_solve_matches_reference(c1):
    from oracle.multibody import gmres
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED
    wl, S, ctx = c1
    v = S.plane_waves(wl.dirs)[:, 0]
    x_ref, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-13)
    vd = ctx.incident_plane_waves(wl.dirs)
    for mode in (SOLVE_FP64, SOLVE_MIXED):
        sol, info = ctx.solve(vd, mode=mode, tol=1e-11)
        err = np.linalg.norm(sol.cpu().numpy()[0] - x_ref) / np.linalg.norm(x_ref)
        print(f"mode {mode}: {info[0]} err {err:.2e} (reference iterations {it})")
        assert err < 1e-8


# --------------------------------------------------------------------------
# uneven bodies, many right-hand sides: 3 spheres, 3 spheroids, 2 bowls
# (kappa = 2 pi, N = 16,810, 64 plane waves on a Fibonacci sphere)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mixed():
    from oracle.multibody import System
    from workloads import configs
    wl = configs.mixed_bodies()
    print(f"[gpu] building context for {wl.name} N={wl.N}", flush=True)
    return wl, System.from_workload(wl), _ctx_for(wl)


def test_mixed_bodies_modal_matrices(mixed):
    wl, S, ctx = mixed
    seen = set()
    for bid, body in enumerate(S.bodies):
        sh = body.shape
        if id(sh) in seen:
            continue
        seen.add(id(sh))
        e = rel(ctx.modal_matrices(bid, 0, sh.M, sh.NG).cpu().numpy(), sh.modal_matrices())
        es = rel(ctx.modal_matrices(bid, 1, sh.M, sh.NG).cpu().numpy(), sh.inverses())
        print(f"body {bid} ({wl.bodies[bid].contour.kind}, NG={sh.NG}): A~ {e:.2e} S {es:.2e}")
        tol = COARSE_SPHEROID_TOL if wl.bodies[bid].contour.kind == "prolate" else MODAL_TOL
        assert e < tol and es < tol


def test_mixed_bodies_operator_64_rhs(mixed):
    """All 64 right-hand sides in one call; the reference checks three of them."""
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = mixed
    sig = _rand(S.N, 64, 61)
    picks = [0, 37, 63]
    ref = np.stack([S.matvec(sig[c]) for c in picks])
    for prec, tol in ((FP64, FP64_TOL), (FP32, fp32_sum_bound(wl))):
        y = ctx.apply_matvec(_dev(sig), prec).cpu().numpy()[picks]
        e = rel(y, ref)
        print(f"prec {prec}: rel err {e:.2e}")
        assert e < tol, e


def test_mixed_bodies_batched_solve_is_certified_by_reference(mixed):
    """64 plane waves solved in one batched mixed-precision solve; the reference
    operator certifies the residual of sampled right-hand sides."""
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = mixed
    v = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-9, max_iters=100)
    print(f"outer {[i['iterations'] for i in info][:4]}... inner {info[0]['inner_iterations']}")
    assert all(i["converged"] for i in info)
    x = sol.cpu().numpy()
    vv = S.plane_waves(wl.dirs)
    for c in (0, 21, 63):
        b = S.rhs(vv[:, c])
        r = np.linalg.norm(b - S.matvec(x[c])) / np.linalg.norm(b)
        print(f"rhs {c}: reference residual {r:.2e} (library {info[c]['rel_residual']:.2e})")
        assert r < 3e-9


def test_autotuner_choice_is_valid(small, tmp_path):
    from paper_1406_0236_amd import FP32, autotune
    wl, S, ctx = small
    cfg, timings = autotune.tune(ctx, FP32, 2, ctx.max_nf, cache_path=str(tmp_path / "cache.json"))
    assert len(timings) >= 4 and all(t > 0 for t in timings.values())
    x = _rand(S.N, 2, 71)
    y = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
    assert rel(y, S.apply_B(x.T).T) < fp32_sum_bound(wl)
    # cached: a second call reuses the choice without timing
    cfg2, _ = autotune.tune(ctx, FP32, 2, ctx.max_nf, cache_path=str(tmp_path / "cache.json"))
    assert list(cfg2) == list(cfg)
    ctx.set_interbody_config(FP32, 0, 0, 0, 0)


def test_rhs_groups_fp32_rings(small):
    """37 right-hand sides through 8-, 4- and 1-wide groups (FP32 rings, 128 threads)."""
    from paper_1406_0236_amd import FP32
    wl, S, ctx = small
    sig = _rand(S.N, 37, 81)
    ref = S.apply_B(sig.T).T
    for tpt, splits in ((2, 0), (1, 3)):
        ctx.set_interbody_config(FP32, 2, tpt, 128, splits)
        y = ctx.apply_interbody(_dev(sig), FP32).cpu().numpy()
        e = rel(y, ref)
        print(f"tpt {tpt}: rel err {e:.2e}")
        assert e < fp32_sum_bound(wl), e
    ctx.set_interbody_config(FP32, 0, 0, 0, 0)


def test_mfma_source_order_matches_reference(small):
    """MFMA order: R^2 and n.d from 16x16x4 MFMAs (FP32 and FP64, whose result rows
    differ), 1, 2 or 4 groups of 16 targets per wave, several splits; 3
    right-hand sides (VALU accumulation in groups of 2 and 1)."""
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    x = _rand(S.N, 3, 91)
    ref = S.apply_B(x.T).T
    for prec, tol in ((FP32, fp32_sum_bound(wl)), (FP64, FP64_TOL)):
        for g, splits in ((1, 1), (2, 3), (4, 0), (2, 16)):
            ctx.set_interbody_config(prec, 3, g, 256, splits)
            y = ctx.apply_interbody(_dev(x), prec).cpu().numpy()
            e = rel(y, ref)
            print(f"prec {prec} G {g} splits {splits}: rel err {e:.2e}")
            assert e < tol, (prec, g, splits, e)
        ctx.set_interbody_config(prec, 0, 0, 0, 0)


def test_mfma_accumulation_16_wide(small):
    """37 right-hand sides: two 16-wide groups with the complex multiply-accumulate
    on MFMA, then VALU groups of 4 and 1; every column against the reference,
    and the same result bit for bit on a second call; FP32 and FP64."""
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = small
    x = _rand(S.N, 37, 92)
    ref = S.apply_B(x.T).T
    for prec, tol in ((FP32, fp32_sum_bound(wl)), (FP64, FP64_TOL)):
        for g in (1, 2, 4):
            ctx.set_interbody_config(prec, 3, g, 256, 0)
            y = ctx.apply_interbody(_dev(x), prec).cpu().numpy()
            e = rel(y, ref)
            print(f"prec {prec} G {g}: rel err {e:.2e}")
            assert e < tol, (prec, g, e)
            y2 = ctx.apply_interbody(_dev(x), prec).cpu().numpy()
            assert np.array_equal(y, y2)
        ctx.set_interbody_config(prec, 0, 0, 0, 0)


def test_fp16_multiply_accumulate_matches_reference(small):
    """MFMA order with the complex multiply-accumulate on the FP16 matrix cores
    (kernel values and densities split into scaled high and low FP16 parts):
    37 right-hand sides = two groups of 16 in 32-node source blocks (the last
    block of each body padded) and a remainder of 5 through the FP32 MFMA
    order; 1, 2 or 4 groups of 16 targets per wavefront, several splits; every
    column against the reference to the FP32 tolerance, bit for bit again on a
    second call, and within 2e-6 of the FP32 MFMA order.  It is the library
    default for FP32 from 16 rhs, and refused in FP64."""
    from paper_1406_0236_amd import FP32, FP64, AxsError
    wl, S, ctx = small
    assert ctx.interbody_launch_shape(FP32, 16)[0] == 4
    assert ctx.interbody_launch_shape(FP32, 15)[0] != 4
    x = _rand(S.N, 37, 94)
    ref = S.apply_B(x.T).T
    ctx.set_interbody_config(FP32, 3, 2, 256, 0)
    y3 = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
    for g, splits in ((1, 0), (2, 3), (4, 16)):
        ctx.set_interbody_config(FP32, 4, g, 256, splits)
        y = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
        e, e3 = rel(y, ref), rel(y, y3)
        print(f"G {g} splits {splits}: rel err {e:.2e}, vs FP32 MFMA order {e3:.2e}")
        assert e < fp32_sum_bound(wl, 16) and e3 < 2e-6, (g, splits, e, e3)
        assert np.array_equal(y, ctx.apply_interbody(_dev(x), FP32).cpu().numpy())
    ctx.set_interbody_config(FP32, 0, 0, 0, 0)
    ctx.set_interbody_config(FP64, 4, 2, 256, 0)
    with pytest.raises(AxsError, match="EINVAL"):
        ctx.apply_interbody(_dev(x[:16]), FP64)
    ctx.set_interbody_config(FP64, 0, 0, 0, 0)


def test_fp16_multiply_accumulate_scales_each_rhs(small):
    """Per-rhs density scales: 16 columns whose magnitudes run from 1e-30 to 1e+30
    and one zero column; each column relative to its own largest value."""
    from paper_1406_0236_amd import FP32
    wl, S, ctx = small
    x = _rand(S.N, 16, 95) * (10.0 ** np.linspace(-30, 30, 16))[:, None]
    x[7] = 0.0
    ref = S.apply_B(x.T).T
    ctx.set_interbody_config(FP32, 4, 2, 256, 0)
    y = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
    ctx.set_interbody_config(FP32, 0, 0, 0, 0)
    assert np.all(y[7] == 0)
    worst = max(rel(y[c], ref[c]) for c in range(16) if c != 7)
    print(f"worst column rel err {worst:.2e}")
    assert worst < fp32_sum_bound(wl, 16), worst


def _edge_workload(tip_gap):
    """A sphere of 144 nodes (four full 32-node blocks and a ragged one), a
    spheroid of 84 nodes lying along x with its tip `tip_gap` from the sphere,
    and a small sphere of 15 nodes (one padded block)."""
    from workloads import configs, geometry as geo
    to_x = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])   # body z axis -> x
    return configs.Workload(f"fp16_edges_gap{tip_gap}", 3.0, 3.0, [
        configs.BodySpec(geo.sphere(1.0, 4, 4), np.zeros(3), np.eye(3), 4),
        configs.BodySpec(geo.prolate(0.5, 1.0, 3, 4), np.array([2.0 + tip_gap, 0.0, 0.0]), to_x, 3),
        configs.BodySpec(geo.sphere(0.3, 1, 3), np.array([0.0, 2.5, 0.0]), np.eye(3), 2)],
        np.array([[0.0, 0.0, 1.0]]))


def test_fp16_multiply_accumulate_ragged_blocks():
    """Ragged and padded 32-node source blocks (bodies of 144, 84 and 15
    nodes; the spheroid's tip 0.3 from the sphere) with 16, 17 and 33 rhs (one
    or two full groups; remainders through the FP32 MFMA order), 1, 2 and 4
    target groups per wavefront: every column against the reference to the
    FP32 tolerance and within 2e-6 of the FP32 MFMA order."""
    from oracle.multibody import System
    from paper_1406_0236_amd import FP32
    wl = _edge_workload(0.3)
    assert [b.n_nodes for b in wl.bodies] == [144, 84, 15]
    S = System.from_workload(wl)
    ctx = _ctx_for(wl)
    try:
        assert ctx.interbody_launch_shape(FP32, 16)[0] == 4
        for nrhs, seed in ((16, 96), (17, 97), (33, 98)):
            x = _rand(S.N, nrhs, seed)
            ref = S.apply_B(x.T).T
            ctx.set_interbody_config(FP32, 3, 2, 256, 0)
            y3 = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
            for g in (1, 2, 4):
                ctx.set_interbody_config(FP32, 4, g, 256, 0)
                y = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
                e = max(rel(y[c], ref[c]) for c in range(nrhs))
                e3 = max(rel(y[c], y3[c]) for c in range(nrhs))
                print(f"{nrhs} rhs, G {g}: worst column rel err {e:.2e}, vs FP32 MFMA order {e3:.2e}")
                assert e < fp32_sum_bound(wl, 16) and e3 < 2e-6, (nrhs, g, e, e3)
    finally:
        ctx.set_interbody_config(FP32, 0, 0, 0, 0)
        ctx.close()


def test_fp16_multiply_accumulate_negative_scale_exponent():
    """The spheroid's tip 0.01 from the sphere: kernel values up to ~1e4, so
    the power of two that brings them into FP16 range is below 1.  The FP16
    multiply-accumulate must agree with the FP32 MFMA order, which shares its
    kernel values.  Both differ from the FP64 reference by more than at wider
    gaps: the MFMA and ring orders form R^2 as |p|^2 - 2 y.p + |y|^2 in the
    source body's frame, which loses about eps32 |p|^2 / R^2 in relative terms
    for pairs this close (the FP64 outer iteration of the mixed solver
    absorbs it); that error is printed and bounded by close_pair_bound."""
    from oracle.multibody import System
    from paper_1406_0236_amd import FP32
    wl = _edge_workload(0.01)
    S = System.from_workload(wl)
    ctx = _ctx_for(wl)
    try:
        x = _rand(S.N, 17, 99)
        ref = S.apply_B(x.T).T
        ctx.set_interbody_config(FP32, 3, 2, 256, 0)
        y3 = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
        ctx.set_interbody_config(FP32, 4, 2, 256, 0)
        y = ctx.apply_interbody(_dev(x), FP32).cpu().numpy()
        e3 = max(rel(y[c], y3[c]) for c in range(17))
        e = max(rel(y[c], ref[c]) for c in range(17))
        print(f"gap 0.01: FP16 vs FP32 MFMA order {e3:.2e}; vs FP64 reference {e:.2e}")
        assert e3 < 2e-6, e3
        bound = close_pair_bound(wl) + fp32_sum_bound(wl, 16)
        print(f"derived bound {bound:.2e}")
        assert e < bound, (e, bound)
    finally:
        ctx.set_interbody_config(FP32, 0, 0, 0, 0)
        ctx.close()


def _low_modes_workload():
    from workloads import configs, geometry as geo
    return configs.Workload("low_modes", 2.0, 2.0, [
        configs.BodySpec(geo.sphere(1.0, 2, 10), np.zeros(3), np.eye(3), 0),
        configs.BodySpec(geo.sphere(0.7, 2, 10), np.array([2.5, 0.3, 0.0]), np.eye(3), 1),
        configs.BodySpec(geo.prolate(0.4, 0.9, 2, 10), np.array([-0.4, 2.6, 0.5]),
                         geo.random_rotation(np.random.default_rng(3)), 2)],
        np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]]))


def test_maximum_rhs_count():
    """The largest batch the ABI accepts, 4096 right-hand sides (256 groups of
    16 in the MFMA order, with the FP16 multiply-accumulate in FP32), on a
    small workload (N = 180): sampled columns of the preconditioned operator
    against the reference, and 4097 refused."""
    from oracle.multibody import System
    from paper_1406_0236_amd import FP32, FP64, AxsError
    wl = _low_modes_workload()
    S = System.from_workload(wl)
    ctx = _ctx_for(wl)
    try:
        x = _rand(S.N, 4096, 91)
        cols = [0, 1, 1000, 2047, 4095]
        ref = np.stack([S.matvec(x[c]) for c in cols])
        xd = _dev(x)
        for prec, tol in ((FP64, FP64_TOL), (FP32, fp32_sum_bound(wl))):
            y = ctx.apply_matvec(xd, prec).cpu().numpy()
            e = rel(y[cols], ref)
            print(f"prec {prec}, 4096 rhs, launch shape {ctx.interbody_launch_shape(prec, 4096)}: "
                  f"sampled columns rel err {e:.2e}")
            assert e < tol
        with pytest.raises(AxsError, match="EINVAL"):
            ctx.apply_matvec(_dev(_rand(S.N, 4097, 92)), FP64)
    finally:
        ctx.close()


def test_lowest_mode_counts():
    """Degenerate azimuthal resolutions: a sphere with M = 0 (one azimuthal node
    per ring, the axisymmetric mode only), a sphere with M = 1 and a rotated
    spheroid with M = 2, side by side (N = 180).  Modal matrices, the
    preconditioned operator in FP64 and FP32 (1 and 17 rhs, every source
    order the context allows) and a solve against the dense reference."""
    from oracle.multibody import System
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED
    wl = _low_modes_workload()
    assert [b.n_nodes for b in wl.bodies] == [20, 60, 100]
    S = System.from_workload(wl)
    ctx = _ctx_for(wl)
    try:
        for bid, body in enumerate(S.bodies):
            sh = body.shape
            e = rel(ctx.modal_matrices(bid, 1, sh.M, sh.NG).cpu().numpy(), sh.inverses())
            print(f"body {bid} ({wl.bodies[bid].contour.kind}, NG={sh.NG}, M={sh.M}): S {e:.2e}")
            tol = COARSE_SPHEROID_TOL if wl.bodies[bid].contour.kind == "prolate" else MODAL_TOL
            assert e < tol, (bid, e)
        for nrhs, seed in ((1, 81), (17, 82)):
            x = _rand(S.N, nrhs, seed)
            ref = np.stack([S.matvec(x[c]) for c in range(nrhs)])
            for prec, tol in ((FP64, 1e-11), (FP32, fp32_sum_bound(wl, 16))):
                for variant in (0, 1, 2, 3):
                    ctx.set_interbody_config(prec, variant, 0, 0, 0)
                    y = ctx.apply_matvec(_dev(x), prec).cpu().numpy()
                    e = rel(y, ref)
                    assert e < tol, (nrhs, prec, variant, e)
                ctx.set_interbody_config(prec, 0, 0, 0, 0)
            print(f"{nrhs} rhs: operator rel err within tolerance for every source order")
        v = S.plane_waves(wl.dirs)
        x_ref = np.stack([S.solve_dense(v[:, c]) for c in range(2)])
        vd = ctx.incident_plane_waves(wl.dirs)
        for mode in (SOLVE_FP64, SOLVE_MIXED):
            sol, info = ctx.solve(vd, mode=mode, tol=1e-11)
            e = rel(sol.cpu().numpy(), x_ref)
            print(f"mode {mode}: solve rel err {e:.2e}")
            assert e < 1e-8
    finally:
        ctx.close()


def test_target_body_range_is_one_gpus_share(mixed):
    """One GPU's share of the block rows (axs_set_target_bodies): the sum over
    all sources for the targets of bodies 2-4 of the 8 mixed bodies, zero
    elsewhere, in FP64 (3 rhs, ring order) and FP32 (16 rhs, FP16
    multiply-accumulate; 5 rhs, ring order).  With the launch shape pinned the
    rows equal the full sum's bit for bit; with the default shape (splits
    chosen for the share) within rounding; the rows against the reference; the
    solves refuse while the range is set, the compressed one included (its
    certificate applies the full operator); (0, 0) restores every row."""
    from paper_1406_0236_amd import FP32, FP64, SOLVE_MIXED, AxsError
    wl, S, ctx = mixed
    ctx.skeletonize(1e-8)   # so that the compressed solve fails on the range, not on a missing skeleton
    lo = sum(b.n_nodes for b in wl.bodies[:2])
    hi = sum(b.n_nodes for b in wl.bodies[:5])
    for prec, nrhs, seed in ((FP64, 3, 71), (FP32, 16, 72), (FP32, 5, 73)):
        x = _dev(_rand(S.N, nrhs, seed))
        full = ctx.apply_interbody(x, prec).cpu().numpy()
        shape = ctx.interbody_launch_shape(prec, nrhs)
        ctx.set_target_bodies(2, 3)
        try:
            part = ctx.apply_interbody(x, prec).cpu().numpy()
            ctx.set_interbody_config(prec, *shape)
            pinned = ctx.apply_interbody(x, prec).cpu().numpy()
            ctx.set_interbody_config(prec, 0, 0, 0, 0)
            with pytest.raises(AxsError, match="ESTATE"):
                ctx.apply_matvec(x, prec)
            with pytest.raises(AxsError, match="target-body range"):
                ctx.solve(ctx.incident_plane_waves(wl.dirs[:1]), mode=SOLVE_MIXED, tol=1e-7)
            with pytest.raises(AxsError, match="target-body range"):
                ctx.solve_skeleton(ctx.incident_plane_waves(wl.dirs[:1]), mode=SOLVE_MIXED, tol=1e-7,
                                   certify=True)
        finally:
            ctx.set_target_bodies(0, 0)
        assert np.array_equal(pinned[:, lo:hi], full[:, lo:hi]), (prec, nrhs)
        assert rel(part[:, lo:hi], full[:, lo:hi]) < (1e-13 if prec == FP64 else 2e-6)
        for y in (part, pinned):
            assert np.all(y[:, :lo] == 0) and np.all(y[:, hi:] == 0)
        ref = S.apply_B(x.cpu().numpy()[:2].T).T
        e = rel(part[:2, lo:hi], ref[:, lo:hi])
        print(f"prec {prec}, {nrhs} rhs, launch shape {ctx.interbody_launch_shape(prec, nrhs)}: "
              f"rows of bodies 2-4 rel err {e:.2e}")
        assert e < (FP64_TOL if prec == FP64 else fp32_sum_bound(wl, 16 if nrhs >= 16 else 0))
    assert np.array_equal(ctx.apply_interbody(x, FP32).cpu().numpy(), ctx.apply_interbody(x, FP32).cpu().numpy())
    with pytest.raises(AxsError, match="EINVAL"):
        ctx.set_target_bodies(7, 2)


def test_mfma_source_order_mixed_bodies_64_rhs(mixed):
    """Rotated spheroids and bowls, 8 bodies of three shapes, 64 right-hand sides
    (four MFMA-accumulated groups of 16); three columns against the reference."""
    from paper_1406_0236_amd import FP32
    wl, S, ctx = mixed
    sig = _rand(S.N, 64, 93)
    picks = [0, 17, 63]
    ref = S.apply_B(sig[picks].T).T
    for variant in (3, 4):
        ctx.set_interbody_config(FP32, variant, 2, 256, 0)
        y = ctx.apply_interbody(_dev(sig), FP32).cpu().numpy()[picks]
        e = rel(y, ref)
        print(f"mixed bodies, MFMA order (variant {variant}), 64 rhs: rel err {e:.2e}")
        assert e < fp32_sum_bound(wl, 16), (variant, e)
    ctx.set_interbody_config(FP32, 0, 0, 0, 0)
