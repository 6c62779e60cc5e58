"""Parity on the largest workload: 64 mixed bodies (spheres, spheroids of aspect
U[1, 3], bowls) in a 24^3 box, kappa = 4 pi, N = 1,351,890, 16 plane waves.

At this size the FP64 reference computes sampled outputs one by one: rows of the
inter-body sum over all 1.35 million sources for 16 right-hand sides (FP32 in
the launch shape the library picks for 16 rhs -- the MFMA order with the
FP16 multiply-accumulate -- and FP64),
and rows of the modal matrices of the bowl and of the most elongated spheroid.
Tolerances as in test_gpu_fullsize.py."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


@pytest.fixture(scope="module")
def many():
    from oracle.multibody import System
    from paper_1406_0236_amd import Context
    from workloads import configs
    wl = configs.mixed_many()
    print(f"[gpu] context {wl.name} N={wl.N} bodies={len(wl.bodies)}", flush=True)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    print("[gpu] precomputed", flush=True)
    return wl, System.from_workload(wl), ctx


def test_c5_interbody_sampled_rows_16_rhs(many):
    from oracle.multibody import apply_B_c
    from paper_1406_0236_amd import FP32, FP64
    wl, S, ctx = many
    assert ctx.interbody_launch_shape(FP32, 16)[0] == 4      # MFMA order, FP16 multiply-accumulate
    rng = np.random.default_rng(201)
    sig = rng.standard_normal((16, S.N)) + 1j * rng.standard_normal((16, S.N))
    rows = np.sort(rng.choice(S.N, 96, replace=False))
    rows[0], rows[-1] = 0, S.N - 1
    ref = apply_B_c(S, sig.T, rows).T                         # (16, rows)
    x = torch.from_numpy(sig).to("cuda:0")
    for prec, tol in ((FP32, 1e-4), (FP64, 1e-12)):
        y = ctx.apply_interbody(x, prec).cpu().numpy()[:, rows]
        e = rel(y, ref)
        print(f"prec {prec}: sampled rows x 16 rhs, rel err {e:.2e}", flush=True)
        assert e < tol, e


def test_c5_modal_matrix_rows(many):
    wl, S, ctx = many
    picks = {}
    for b, bs in enumerate(wl.bodies):
        c = bs.contour
        if c.kind == "bowl" and "bowl" not in picks:
            picks["bowl"] = b
        if c.kind == "prolate":
            if "prolate" not in picks or c.NG > wl.bodies[picks["prolate"]].contour.NG:
                picks["prolate"] = b
    for kind, b in picks.items():
        sh = S.bodies[b].shape
        A = ctx.modal_matrices(b, 0, sh.M, sh.NG).cpu().numpy()
        for i in (0, sh.NG // 3, sh.NG - 1):
            row = sh.modal_row(i) + 0.5 * (np.arange(sh.NG) == i)[None, :]
            e = rel(A[:, i, :], row)
            print(f"{kind} body {b} (NG={sh.NG}, M={sh.M}) row {i}: rel err {e:.2e}", flush=True)
            assert e < 1e-9, e
