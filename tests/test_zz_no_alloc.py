"""The allocation-free operator (axs_apply_matvec_noalloc, scratch in a static
device array) through the C ABI against axs_apply_matvec: the same kernels in
the same launch shape, so the results are equal bit for bit; two calls in a
row per precision, the second with fewer right-hand sides; the first call of
each precision runs before the allocating operator has cached its work table;
sizes beyond the static scratch and the MFMA orders are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_operator_equals_the_allocating_one():
    from paper_1406_0236_amd import FP32, FP64, AxsError, Context
    from workloads import configs
    wl = configs.mixed_bodies(n_dirs=1)
    print(f"[gpu] no-alloc operator on {wl.name}, N={wl.N}", flush=True)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    rng = np.random.default_rng(77)
    try:
        for prec in (FP64, FP32):
            for nrhs in (5, 2):
                x = torch.from_numpy(rng.standard_normal((nrhs, wl.N)) + 1j * rng.standard_normal((nrhs, wl.N)))
                x = x.to("cuda:0")
                got = ctx.apply_matvec_noalloc(x, prec)
                ref = ctx.apply_matvec(x, prec)
                print(f"precision {prec}, {nrhs} rhs: max |difference| "
                      f"{float(torch.max(torch.abs(got - ref))):.1e}", flush=True)
                assert torch.equal(got, ref), (prec, nrhs)
        x16 = torch.zeros((16, wl.N), dtype=torch.complex128, device="cuda:0")
        with pytest.raises(AxsError, match="point and ring orders"):
            ctx.apply_matvec_noalloc(x16, FP32)
        ctx.set_interbody_config(FP64, 2, 0, 0, 0)   # ring order pinned: 64 rhs need more than 256 MiB
        x64 = torch.zeros((64, wl.N), dtype=torch.complex128, device="cuda:0")
        with pytest.raises(AxsError, match="beyond the static"):
            ctx.apply_matvec_noalloc(x64, FP64)
        ctx.set_interbody_config(FP64, 0, 0, 0, 0)
    finally:
        ctx.close()
