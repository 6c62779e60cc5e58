"""The warm-start network and its encoding, through the C ABI, against the FP64
reference MLP (oracle/mlp.py) and the definition of the mode encoding.

Tolerances: FP32 network, so forward outputs within 1e-5 and gradients within
1e-4 of the largest entry; the mode maps are FP64 arithmetic stored in FP32
(relative 1e-6)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


@pytest.fixture(scope="module")
def dev_ctx():
    from paper_1406_0236_amd import Context
    ctx = Context(0)
    yield ctx


def _net(ctx, n_in, width, depth, n_out, seed):
    from oracle import mlp as ref
    from paper_1406_0236_amd import Mlp
    rng = np.random.default_rng(seed)
    sizes = ref.layer_sizes(n_in, width, depth, n_out)
    p = ref.init_params(sizes, rng) + 0.05 * rng.standard_normal(ref.n_params(sizes))
    p = p.astype(np.float32).astype(np.float64)
    net = Mlp(ctx, n_in, width, depth, n_out)
    net.set_params(p)
    return net, p, sizes, rng


@pytest.mark.parametrize("shape", [(4, 16, 2, 6, 5), (4, 64, 4, 300, 100), (4, 96, 3, 70, 257)])
def test_forward_and_gradient_match_reference(dev_ctx, shape):
    from oracle import mlp as ref
    n_in, width, depth, n_out, B = shape
    net, p, sizes, rng = _net(dev_ctx, n_in, width, depth, n_out, 1)
    X = rng.standard_normal((B, n_in)).astype(np.float32)
    T = rng.standard_normal((B, n_out)).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    Y = net.forward(Xd).cpu().numpy()
    Yr, _ = ref.forward(p, sizes, X.astype(np.float64))
    assert rel(Y, Yr) < 1e-5, rel(Y, Yr)
    loss, g = net.gradient(Xd, Td)
    lr_, gr = ref.loss_and_grad(p, sizes, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lr_) <= 1e-5 * abs(lr_)
    e = rel(g.cpu().numpy(), gr)
    print(f"{shape}: forward {rel(Y, Yr):.1e} grad {e:.1e}")
    assert e < 1e-4, e
    net.close()


def test_adam_steps_match_reference(dev_ctx):
    from oracle import mlp as ref
    net, p, sizes, rng = _net(dev_ctx, 4, 32, 2, 12, 2)
    X = rng.standard_normal((40, 4)).astype(np.float32)
    T = rng.standard_normal((40, 12)).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pr = p.copy()
    for t in range(1, 4):
        net.adam_step(Xd, Td, 1e-3)
        _, g = ref.loss_and_grad(pr, sizes, X.astype(np.float64), T.astype(np.float64))
        pr, m, v = ref.adam_step(pr, m, v, g, t, 1e-3)
    got = net.get_params().astype(np.float64)
    assert np.max(np.abs(got - pr)) < 5e-6
    net.close()


def test_train_epoch_matches_steps_one_by_one(dev_ctx):
    """The library's epoch loop (row gather on the device) against the same
    steps taken through axs_mlp_adam_step on batches gathered by the test:
    bitwise equal, and within 5e-6 of the FP64 reference Adam."""
    from oracle import mlp as ref
    from paper_1406_0236_amd import Mlp
    net, p, sizes, rng = _net(dev_ctx, 4, 48, 2, 10, 3)
    twin = Mlp(dev_ctx, 4, 48, 2, 10)
    twin.set_params(p)
    rows = 70
    X = rng.standard_normal((rows, 4)).astype(np.float32)
    T = rng.standard_normal((rows, 10)).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pr = p.copy()
    t = 0
    # 5 steps of 16 (repeated rows, last row included), then 3 of 7
    for batch, steps in ((16, 5), (7, 3)):
        order = rng.integers(0, rows, batch * steps).astype(np.int32)
        order[-1] = rows - 1
        lrs = 1e-3 * (1.0 + np.arange(steps)) / steps
        loss = net.train_epoch(Xd, Td, order, batch, lrs)
        for s in range(steps):
            idx = order[s * batch:(s + 1) * batch]
            il = torch.from_numpy(idx.astype(np.int64)).cuda()
            loss1 = twin.adam_step(Xd.index_select(0, il).contiguous(), Td.index_select(0, il).contiguous(), lrs[s])
            t += 1
            _, g = ref.loss_and_grad(pr, sizes, X[idx].astype(np.float64), T[idx].astype(np.float64))
            pr, m, v = ref.adam_step(pr, m, v, g, t, lrs[s])
        assert loss == loss1
        got = net.get_params()
        assert np.array_equal(got, twin.get_params())
        assert np.max(np.abs(got.astype(np.float64) - pr)) < 5e-6
    twin.close()
    net.close()


def test_train_epoch_rejects_bad_rows_and_rates(dev_ctx):
    from paper_1406_0236_amd import AxsError
    net, p, sizes, rng = _net(dev_ctx, 4, 16, 1, 3, 4)
    Xd = torch.randn(20, 4, device="cuda")
    Td = torch.randn(20, 3, device="cuda")
    before = net.get_params()
    ok = np.arange(8, dtype=np.int32)
    for order, lrs in ((np.array([0, 1, 2, 20], np.int32), [1e-3]), (np.array([0, -1, 2, 3], np.int32), [1e-3]),
                       (ok, [1e-3, 0.0])):
        with pytest.raises(AxsError):
            net.train_epoch(Xd, Td, order, 4, lrs)
    assert np.array_equal(net.get_params(), before)
    net.close()


def test_mode_encoding_matches_its_definition(small_system):
    """c_{b,i,m} = e^{-i k d.c_b} (1/N_F) sum_l sigma e^{-i m th_l}, and decoding
    band-limited densities gives them back."""
    from paper_1406_0236_amd import Context, density_from_modes, modes_from_density
    wl, S = small_system
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    mmax = 5
    rng = np.random.default_rng(3)
    dirs = rng.standard_normal((2, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    sig = rng.standard_normal((2, S.N)) + 1j * rng.standard_normal((2, S.N))
    got = modes_from_density(ctx, torch.from_numpy(sig).cuda(), dirs, mmax).cpu().numpy()
    expect = []
    for c in range(2):
        parts = []
        for b, o0 in zip(S.bodies, S.offsets[:-1]):
            sh = b.shape
            blk = sig[c, o0:o0 + sh.NG * sh.NF].reshape(sh.NG, sh.NF)
            F = np.fft.fft(blk, axis=1) / sh.NF
            ph = np.exp(-1j * wl.kappa * dirs[c] @ b.centre)
            m = np.arange(-mmax, mmax + 1)
            co = F[:, m % sh.NF] * ph
            parts.append(np.stack([co.real, co.imag], axis=-1).ravel())
        expect.append(np.concatenate(parts))
    expect = np.array(expect)
    assert rel(got, expect) < 1e-6
    # band-limited density -> modes -> density
    back = density_from_modes(ctx, torch.from_numpy(got).cuda(), dirs, mmax).cpu().numpy()
    again = modes_from_density(ctx, torch.from_numpy(back).cuda(), dirs, mmax).cpu().numpy()
    assert rel(again, got) < 1e-6
    ctx.close()


def test_learned_warm_start_gain_small():
    """Train on the mixed-body geometry (reduced: 12 wavenumbers x 32 directions),
    evaluate on held-out wavenumbers; the guess must not cost iterations on
    average, and the numbers are printed."""
    from paper_1406_0236_amd import Context, warm_start_size
    from paper_1406_0236_amd import warmstart as W
    from workloads import configs
    wl_at = lambda k: configs.mixed_bodies(kappa=k, disc_kappa=W.K_MAX, n_dirs=1)
    rng = np.random.default_rng(4)
    ks = rng.uniform(W.K_MIN, W.K_MAX, 12)
    dirs = [W.random_directions(32, rng) for _ in ks]
    X, Y = W.generate(wl_at, ks, dirs, mmax=8, tol=1e-8, log=print)
    dev = Context(0)
    ws = W.WarmStart(dev, Y.shape[1], mmax=8, width=256, depth=4)
    hist = ws.train(X, Y, epochs=150, batch=64, lr=1e-3, log=print)
    assert hist[-1] < 0.5 * hist[0]
    rng2 = np.random.default_rng(40)
    hk = rng2.uniform(W.K_MIN, W.K_MAX, 2)
    hd = [W.random_directions(16, rng2) for _ in hk]
    rows = W.evaluate(ws, wl_at, hk, hd, tol=1e-7, log=print)
    zero = np.mean([r["fp64"]["zero_iters"] for r in rows])
    warm = np.mean([r["fp64"]["warm_iters"] for r in rows])
    print(f"held-out FP64 GMRES iterations: zero guess {zero:.2f}, learned guess {warm:.2f}")
    assert all(r["fp64"]["converged"] and r["mixed"]["converged"] for r in rows)
    assert warm <= zero + 0.5
