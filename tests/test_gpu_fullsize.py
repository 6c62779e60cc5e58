"""Parity at the benchmark's full size (27 spheres, kappa = 4 pi, N = 437,400) and
in the launch configuration bench.py times (library defaults), on outputs the
FP64 reference can compute one by one: sampled rows of the inter-body sum,
sampled rows of the modal matrices, and the residual of the solve on the rows of one
body (on every row with AXS_CERTIFY_EVERY_ROW=1).  Tolerances as in test_gpu_parity.py; the FP32 bound is
looser here (phases reach kappa R ~ 200 rad, so FP32 coordinates give
kappa |x| 2^-24 ~ 4e-6 rad per pair)."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from tolerances import fp32_sum_bound  # noqa: E402


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


@pytest.fixture(scope="module")
def lattice():
    from oracle.multibody import System
    from paper_1406_0236_amd import Context
    from workloads import configs
    wl = configs.sphere_lattice()
    print(f"[gpu] full-size context {wl.name} N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return wl, System.from_workload(wl), ctx


def test_fullsize_interbody_sampled_rows(lattice):
    from oracle.multibody import apply_B_c
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = lattice
    rng = np.random.default_rng(101)
    sig = rng.standard_normal(S.N) + 1j * rng.standard_normal(S.N)
    rows = np.sort(rng.choice(S.N, 256, replace=False))
    rows[0], rows[-1] = 0, S.N - 1          # first and last node (ragged tile ends)
    ref = apply_B_c(S, sig, rows)
    x = torch.from_numpy(sig[None]).to("cuda:0")
    for prec, tol in ((FP64, 4e-13), (FP32, fp32_sum_bound(wl))):
        y = ctx.apply_interbody(x, prec).cpu().numpy()[0][rows]
        e = rel(y, ref)
        print(f"prec {prec}: sampled-row rel err {e:.2e}")
        assert e < tol, e


def test_fullsize_modal_matrix_rows(lattice):
    wl, S, ctx = lattice
    sh = S.bodies[0].shape
    A = ctx.modal_matrices(0, 0, sh.M, sh.NG).cpu().numpy()
    for i in (0, 57, 103, 199):
        row = sh.modal_row(i) + 0.5 * (np.arange(sh.NG) == i)[None, :]
        e = rel(A[:, i, :], row)
        print(f"row {i}: rel err {e:.2e}")
        assert e < 2e-12, e


def _certified_residual(S, wl, x, rows_of, log_every=None):
    """The reference's residual x + D^{-1} B x - b, b = -D^{-1} v, on the rows of
    the bodies in rows_of (its own inter-body sum over every source, per-mode
    inverses and plane wave), and ||b|| over the same bodies."""
    import time
    from oracle.multibody import apply_B_c
    vr = S.plane_waves(wl.dirs)[:, 0]
    r2 = b2 = 0.0
    t0 = time.time()
    for n, b_id in enumerate(rows_of):
        o0, o1 = S.offsets[b_id], S.offsets[b_id + 1]
        sh = S.bodies[b_id].shape
        Bx = apply_B_c(S, x, np.arange(o0, o1))
        bb = -sh.apply_Ainv(vr[o0:o1].reshape(sh.NG, sh.NF)).reshape(-1)
        r = x[o0:o1] + sh.apply_Ainv(Bx.reshape(sh.NG, sh.NF)).reshape(-1) - bb
        r2 += float(np.vdot(r, r).real)
        b2 += float(np.vdot(bb, bb).real)
        if log_every and (n + 1) % log_every == 0:
            print(f"[gpu] reference residual: {n + 1} of {len(rows_of)} bodies, {time.time() - t0:.0f} s", flush=True)
    return math.sqrt(r2), math.sqrt(b2)


def test_fullsize_solve_residual_certified_on_one_body(lattice):
    """Mixed solve to 1e-7 as in the benchmark; the reference recomputes the
    residual on all rows of body 13 (the centre), relative to the library's
    ||b|| over all rows."""
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = lattice
    v = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-7)
    print(info[0])
    assert info[0]["converged"]
    rn, _ = _certified_residual(S, wl, sol.cpu().numpy()[0], [13])
    e = rn / float(torch.linalg.norm(ctx.apply_precond(v)))
    print(f"body 13: reference residual {e:.2e} (library total {info[0]['rel_residual']:.2e})")
    assert e <= 1e-7


@pytest.mark.slow
@pytest.mark.timeout(1200)
@pytest.mark.skipif(os.environ.get("AXS_CERTIFY_EVERY_ROW") != "1",
                    reason="4-7 minutes of host time on 16 threads (1.8e11 reference kernel evaluations): "
                           "run with AXS_CERTIFY_EVERY_ROW=1")
def test_fullsize_solve_residual_certified_on_every_row(lattice):
    """Mixed solve to 1e-7 as in the benchmark; the reference recomputes the
    residual x + D^{-1} B x - b on all 437,400 rows: its relative residual is
    within the tolerance and equals the library's explicit FP64 residual to
    1e-10 (the two operators agree to about 1e-13 on these well-conditioned
    spheres)."""
    from oracle.multibody import num_threads
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = lattice
    v = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-7, certify=True)
    print(info[0], flush=True)
    assert info[0]["converged"]
    print(f"[gpu] reference inter-body sum on all {S.N} rows, {num_threads()} threads", flush=True)
    rn, bn = _certified_residual(S, wl, sol.cpu().numpy()[0], list(range(len(S.bodies))), log_every=1)
    e = rn / bn
    print(f"every row: reference residual {e:.3e}, library explicit residual {info[0]['rel_residual']:.3e}")
    assert e <= 1e-7 * (1 + 1e-3)
    assert abs(e - info[0]["rel_residual"]) < 1e-10


def test_fullsize_augmented_inner_runs_save_iterations(lattice):
    """On the 27 spheres the second inner run, augmented with the first one's
    Krylov space, needs fewer FP32 iterations than one restarted from scratch,
    with the same number of outer steps and both answers certified."""
    from paper_1406_0236_amd import SOLVE_MIXED, SOLVE_RESTART_INNER
    wl, S, ctx = lattice
    v = ctx.incident_plane_waves(wl.dirs)
    res = {}
    for name, mode in (("augmented", SOLVE_MIXED), ("restarted", SOLVE_MIXED | SOLVE_RESTART_INNER)):
        sol, info = ctx.solve(v, mode=mode, tol=1e-7, certify=True)
        print(name, info[0])
        assert info[0]["converged"]
        res[name] = info[0]
    assert res["augmented"]["iterations"] == res["restarted"]["iterations"]
    assert res["augmented"]["inner_iterations"] < res["restarted"]["inner_iterations"]


def test_fullsize_skeleton_solve(lattice):
    """The benchmark problem through the ring skeletonization (Sec. 5, eps = 1e-8):
    the ring rank equals the reference's ID of the same shape and proxy sphere
    (within 2), and the lifted density of a mixed solve to 1e-7 has a full-system
    FP64 residual below 1e-7 and agrees with the uncompressed mixed solution to
    the solve tolerance."""
    from oracle.nystrom import Shape
    from oracle.skeleton import ring_id
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = lattice
    ns = ctx.skeletonize(1e-8, 2.0)
    k, ng = ctx.skeleton_rank(0)
    c = wl.bodies[0].contour
    sh = Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, wl.kappa, wl.eta, wl.bodies[0].M)
    kr = ring_id(sh, 2.0, 1e-8)[1].shape[1]
    print(f"rings {k} of {ng} (reference {kr}), {ns} of {wl.N} unknowns", flush=True)
    assert abs(k - kr) <= 2 and ns == 27 * k * sh.NF
    v = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=1e-7, certify=True)
    ref, _ = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-7)
    d = float(torch.linalg.norm(sol - ref) / torch.linalg.norm(ref))
    print(f"skeleton solve: {info[0]['iterations']} outer, {info[0]['inner_iterations']} inner, "
          f"full residual {info[0]['rel_residual']:.2e}, vs uncompressed {d:.2e}")
    assert info[0]["rel_residual"] < 1e-7
    assert d < 1e-6


def test_fullsize_point_skeleton_solve(lattice):
    """The benchmark problem through point skeletons (the randomized ID of single
    nodes, eps = 1e-10): fewer than a fifth of the nodes stay, and the lifted
    density of a mixed solve to 1e-7 has a full-system residual below 1e-7, by
    the library's FP64 certificate on every row and by the reference's own
    residual on the rows of body 13 (relative to the library's ||b||), and
    agrees with the uncompressed mixed solution to 1e-6."""
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = lattice
    ns = ctx.skeletonize_points(1e-10, 2.0, 0, 1)
    k, n = ctx.skeleton_rank(0)
    print(f"point skeletons: {k} of {n} nodes per body, {ns} of {wl.N} unknowns", flush=True)
    assert ns == 27 * k and k < 0.2 * n
    v = ctx.incident_plane_waves(wl.dirs)
    sol, info = ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=1e-7, certify=True)
    ref, _ = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-7)
    d = float(torch.linalg.norm(sol - ref) / torch.linalg.norm(ref))
    rn, _ = _certified_residual(S, wl, sol.cpu().numpy()[0], [13])
    e = rn / float(torch.linalg.norm(ctx.apply_precond(v)))
    print(f"point skeleton solve: {info[0]['iterations']} outer, {info[0]['inner_iterations']} inner, "
          f"full residual {info[0]['rel_residual']:.2e}, body 13 by the reference {e:.2e}, "
          f"vs uncompressed {d:.2e}", flush=True)
    assert info[0]["rel_residual"] < 1e-7 and e < 1e-7
    assert d < 1e-6


def test_fullsize_point_id_interpolates_unseen_fields(lattice):
    """The point ID of the 27-sphere shape (eps 1e-10, 16,200 nodes) against
    fields it never saw, computed here from their definitions: point sources
    outside its proxy sphere (incoming; the ID must reproduce u from u(I)) and
    a random density's field at far targets (outgoing; A_far X^T sigma on the
    skeleton nodes).  Both to 5e-8 (1.9e-9 and 2.3e-9 seen)."""
    wl, S, ctx = lattice
    ctx.skeletonize_points(1e-10, 2.0, 0, 1)
    nodes = ctx.skeleton_nodes(0)
    XT = ctx.skeleton_interp(0).cpu().numpy()                 # k x n
    body = S.bodies[0]
    n = body.shape.NG * body.shape.NF
    assert XT.shape == (nodes.size, n)
    rng = np.random.default_rng(41)
    d = rng.standard_normal((12, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    src = d * rng.uniform(2.1, 4.0, 12)[:, None]              # the proxy radius is 2 here
    loc = body.x - body.centre
    R = np.linalg.norm(loc[:, None, :] - src[None, :, :], axis=-1)
    u = (np.exp(1j * wl.kappa * R) / (4 * np.pi * R)) @ rng.standard_normal(12)
    e_in = np.linalg.norm(XT.T @ u[nodes] - u) / np.linalg.norm(u)
    tg = body.centre + 3.0 * d
    sig = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    G = S.kernel(tg, body.x, body.n) * S.w[:n][None, :]
    e_out = np.linalg.norm(G[:, nodes] @ (XT @ sig) - G @ sig) / np.linalg.norm(G @ sig)
    print(f"point ID of the 27-sphere shape: {nodes.size} of {n} nodes; unseen incoming {e_in:.2e}, "
          f"outgoing {e_out:.2e}", flush=True)
    assert e_in < 5e-8 and e_out < 5e-8


def test_fullsize_reciprocity(lattice):
    """At the benchmark's full size (27 spheres, N = 437,400, kappa = 4 pi): two
    incident directions d1, d2 solved in one batched mixed solve to 1e-9;
    reciprocity u_inf(x^ = -d2; d1) = u_inf(x^ = -d1; d2) of their far fields.
    A property of the exact solution; the discrete one keeps it to 1e-9."""
    from paper_1406_0236_amd import SOLVE_MIXED
    wl, S, ctx = lattice
    d = np.array([[0.0, 0.6, 0.8], [0.48, -0.6, 0.64]])
    v = ctx.incident_plane_waves(d)
    sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-9)
    assert all(i["converged"] for i in info)
    u12 = ctx.far_field(sol[:1].contiguous(), -d[1:2]).cpu().numpy()[0, 0]
    u21 = ctx.far_field(sol[1:2].contiguous(), -d[0:1]).cpu().numpy()[0, 0]
    e = abs(u12 - u21) / max(abs(u12), abs(u21))
    print(f"full size reciprocity: {e:.2e} ({info[0]['iterations']} outer, {info[0]['inner_iterations']} inner)")
    assert e < 1e-7   # seen 1.1e-9


def test_fullsize_greens_identity():
    """The paper's accuracy protocol (Sec. 6) at the benchmark's full size: one
    point source inside each of the 27 spheres, the incident field their
    field, a mixed solve to 1e-9, and the scattered field at 10 exterior
    targets against the exact one (minus the sources' field)."""
    import math
    from paper_1406_0236_amd import SOLVE_MIXED, Context
    from workloads import configs
    wl = configs.sphere_lattice()
    ctx = Context(0).add_workload(wl)
    try:
        ctx.precompute_scattering()
        src = configs.point_sources(wl, seed=11)
        amp = np.random.default_rng(12).standard_normal(len(src))
        v = ctx.incident_point_sources(src, amp)
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=1e-9)
        assert info[0]["converged"]
        xt = configs.exterior_targets(wl, 10, seed=12)
        u = ctx.eval_field(sol, xt).cpu().numpy()[0]
        dist = np.linalg.norm(xt[:, None, :] - src[None, :, :], axis=-1)
        exact = -(np.exp(1j * wl.kappa * dist) / (4.0 * math.pi * dist)) @ amp
        e = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
        print(f"full size Green's identity: E_inf {e:.2e}")
        assert e < 1e-8   # seen 4.0e-10
    finally:
        ctx.close()
