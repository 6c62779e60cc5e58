"""The warm-start network and its encoding, through the C ABI, against the FP64
reference MLP (oracle/mlp.py) and the definition of the encoding (the
reference's inter-body sum and per-body inverses).

Tolerances: FP32 network, so forward outputs within 1e-5 and gradients within
1e-4 of the largest entry; the encoding is FP64 arithmetic stored in FP32
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


# -- the library's training loop against the reference --------------------------------
_MASK = (1 << 64) - 1


def _splitmix64(x):
    x = (x + 0x9E3779B97F4A7C15) & _MASK
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _MASK
    return x ^ (x >> 31)


def _uniform01(seed, k):
    """The counter-based uniform draw axs_mlp_train documents (splitmix64 of seed, counter)."""
    return (float(_splitmix64((seed * 0x632BE59BD9B4E019 + k) & _MASK) >> 11) + 0.5) * (1.0 / 9007199254740992.0)


def test_train_matches_reference_steps(dev_ctx):
    """axs_mlp_train (feature scaling, target scaling, seeded permutations, cosine
    learning rate, Adam, the scale folded into the last layer) against the same
    schedule run by the FP64 reference MLP: per-epoch losses and parameters."""
    from oracle import mlp as ref
    from paper_1406_0236_amd import mlp_train
    n_out, S, batch, epochs = 6, 40, 8, 3
    net, p, sizes, rng = _net(dev_ctx, 4, 16, 2, n_out, 11)
    X = np.concatenate([rng.standard_normal((S, 3)), rng.uniform(4.0, 8.0, (S, 1))], axis=1).astype(np.float32)
    Y = (3.0 * rng.standard_normal((S, n_out))).astype(np.float32)
    kmin, kmax, seed, lr0, lr1 = 4.0, 8.0, 9, 2e-3, 1e-4
    losses = mlp_train(net, torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                       {"epochs": epochs, "batch": batch, "lr": lr0, "lr_final": lr1, "seed": seed,
                        "init_seed": -1, "k_min": kmin, "k_max": kmax})
    got = net.get_params().astype(np.float64)
    # the reference schedule
    scale = math.sqrt(np.mean(Y.astype(np.float64) ** 2))
    Xs = X.astype(np.float64).copy()
    Xs[:, 3] = ((2.0 * X[:, 3].astype(np.float64) - (kmin + kmax)) / (kmax - kmin)).astype(np.float32)
    Ys = (Y * np.float32(1.0 / scale)).astype(np.float64)
    last = sum(a * b + b for a, b in zip(sizes[:-2], sizes[1:-1]))
    pr = p.copy()
    pr[last:] = (p[last:].astype(np.float32) * np.float32(1.0 / scale)).astype(np.float64)
    m, v = np.zeros_like(pr), np.zeros_like(pr)
    steps = S // batch
    total = epochs * steps
    draw, t = 0, 0
    for ep in range(epochs):
        perm = list(range(S))
        for i in range(S - 1, 0, -1):
            j = min(int(_uniform01(seed, draw) * (i + 1)), i)
            draw += 1
            perm[i], perm[j] = perm[j], perm[i]
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * (ep * steps + s) / (total - 1)))
            loss, g = ref.loss_and_grad(pr, sizes, Xs[idx], Ys[idx])
            t += 1
            pr, m, v = ref.adam_step(pr, m, v, g, t, lr)
        assert abs(losses[ep] - loss) <= 1e-5 * abs(loss), (ep, losses[ep], loss)
    pr[last:] *= scale
    e = np.max(np.abs(got - pr)) / np.max(np.abs(pr))
    print(f"train: {epochs} epochs x {steps} steps, parameters within {e:.1e} of the reference")
    assert e < 2e-5, e
    net.close()


def test_train_he_initialisation_and_bad_hparams(dev_ctx):
    """init_seed >= 0 draws W ~ N(0, 2 / fan_in) (Box-Muller on the documented
    counter-based uniforms) with zero biases; malformed or incomplete hparams
    are refused before anything changes."""
    from oracle import mlp as ref
    from paper_1406_0236_amd import AxsError, mlp_train
    net, p, sizes, rng = _net(dev_ctx, 4, 8, 1, 3, 12)
    X = torch.randn(8, 4, device="cuda")
    Y = torch.randn(8, 3, device="cuda")
    before = net.get_params()
    for hp in ({"epochs": 1}, {"k_min": 2.0, "k_max": 1.0}, {"k_min": 1.0, "k_max": 2.0, "lr": 0.0},
               {"k_min": 1.0, "k_max": 2.0, "momentum": 0.5}):
        with pytest.raises(AxsError, match="EINVAL"):
            mlp_train(net, X, Y, hp)
    for text in (b"[1, 2]", b'{"k_min": 1, "k_max": 2', b'{"k_min": "a", "k_max": 2}', b'{"k_min": 1, "k_max": 2} x'):
        st = net.lib.axs_mlp_train(net.h, ctypes_ptr(X), ctypes_ptr(Y), 8, text, None)
        assert st == -1, (text, st)
    assert np.array_equal(net.get_params(), before)
    # one epoch at a negligible rate from the He initialisation: the weights are the draws
    seed = 21
    mlp_train(net, X, Y, {"epochs": 1, "batch": 8, "lr": 1e-30, "lr_final": 1e-30, "init_seed": seed,
                          "k_min": 1.0, "k_max": 2.0})
    got = net.get_params().astype(np.float64)
    k = 0
    off = 0
    expect = np.zeros_like(got)
    for a, b in zip(sizes[:-1], sizes[1:]):
        for e in range(a * b):
            u1, u2 = _uniform01(seed, k), _uniform01(seed, k + 1)
            k += 2
            expect[off + e] = np.float32(math.sqrt(2.0 / a) * math.sqrt(-2.0 * math.log(u1)) * math.cos(2 * math.pi * u2))
        off += a * b + b
    last = sum(a * b + b for a, b in zip(sizes[:-2], sizes[1:-1]))
    assert np.max(np.abs(got[:last] - expect[:last])) <= 1e-6 * np.max(np.abs(expect))
    # the target scale (root mean square of Y) is folded into the last layer at the end
    scale = math.sqrt(np.mean(Y.cpu().numpy().astype(np.float64) ** 2))
    assert np.max(np.abs(got[last:] - scale * expect[last:])) <= 1e-6 * scale * np.max(np.abs(expect))
    net.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


# -- the encoding of the learned part -------------------------------------------------
@pytest.fixture(scope="module")
def three_bodies():
    """Sphere, rotated spheroid and rotated bowl at kappa = 2 (three bodies, so the
    source slots s < b and s >= b both occur)."""
    from oracle.multibody import System
    from workloads import configs, geometry as geo
    rng = np.random.default_rng(5)
    k = 2.0
    wl = configs.Workload("three", k, k, [
        configs.BodySpec(geo.sphere(1.0, 4, 10), np.array([0.0, 0.0, 0.0]), np.eye(3), 8),
        configs.BodySpec(geo.prolate(0.8, 1.3, 5, 10), np.array([2.8, 0.4, -0.3]), geo.random_rotation(rng), 7),
        configs.BodySpec(geo.bowl(3, 2, 4, 10), np.array([-0.6, 2.7, 0.5]), geo.random_rotation(rng), 6)],
        geo.fibonacci_directions(3))
    return wl, System.from_workload(wl)


def _ctx(wl):
    from paper_1406_0236_amd import Context
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return ctx


def test_warm_start_encoding_matches_its_definition(three_bodies):
    """Y[b][s][i][m] = e^{-i phi} (1/N_F) sum_l u(i, l) e^{-i m th_l} with
    u = -D_b^{-1} B_{bb'} x_{b'} from the reference's inter-body sum and per-body
    inverses, phi = kappa (d.c_{b'} + |c_b - c_{b'}|); and with every mode kept,
    decode(encode(x)) = -D^{-1} B x from the library's own operator."""
    from paper_1406_0236_amd import FP64, warm_start_decode, warm_start_encode, warm_start_size
    wl, S = three_bodies
    ctx = _ctx(wl)
    rng = np.random.default_rng(8)
    dirs = wl.dirs
    x = rng.standard_normal((3, S.N)) + 1j * rng.standard_normal((3, S.N))
    mmax = 4
    Y = warm_start_encode(ctx, torch.from_numpy(x).cuda(), dirs, mmax).cpu().numpy()
    nb = len(S.bodies)
    assert Y.shape == (3, 2 * (nb - 1) * (2 * mmax + 1) * sum(b.shape.NG for b in S.bodies))
    expect = np.zeros_like(Y)
    m = np.arange(-mmax, mmax + 1)
    for c in range(3):
        off = 0
        for b, body in enumerate(S.bodies):
            sh = body.shape
            o0, o1 = S.offsets[b], S.offsets[b + 1]
            for s in range(nb - 1):
                bs = s if s < b else s + 1
                xm = np.zeros(S.N, dtype=complex)
                xm[S.offsets[bs]:S.offsets[bs + 1]] = x[c, S.offsets[bs]:S.offsets[bs + 1]]
                u = -sh.apply_Ainv(S.apply_B(xm)[o0:o1].reshape(sh.NG, sh.NF))
                phi = wl.kappa * (dirs[c] @ S.bodies[bs].centre + np.linalg.norm(body.centre - S.bodies[bs].centre))
                co = (np.fft.fft(u, axis=1) / sh.NF)[:, m % sh.NF] * np.exp(-1j * phi)
                blk = np.stack([co.real, co.imag], axis=-1).ravel()
                expect[c, off:off + blk.size] = blk
                off += blk.size
    e = rel(Y, expect)
    print(f"encoding vs its definition: {e:.2e}")
    assert e < 1e-6, e
    # all modes: the sum over the sources is exact
    mfull = min(b.M for b in wl.bodies)
    xd = torch.from_numpy(x).cuda()
    Yf = warm_start_encode(ctx, xd, dirs, mfull)
    got = warm_start_decode(ctx, Yf, dirs, mfull).cpu().numpy()
    want = (xd - ctx.apply_matvec(xd, FP64)).cpu().numpy()       # -D^{-1} B x
    # every body's own modes above the common cutoff are lost in the encoding; the
    # bodies with M equal to the cutoff are exact
    for b, body in enumerate(wl.bodies):
        o0, o1 = S.offsets[b], S.offsets[b + 1]
        if body.M == mfull:
            eb = rel(got[:, o0:o1], want[:, o0:o1])
            print(f"body {b}: decode(encode(x)) vs -D^-1 B x: {eb:.2e}")
            assert eb < 1e-6, eb
    assert warm_start_size(ctx, mmax) == Y.shape[1]
    ctx.close()


def test_predict_is_single_body_response_plus_decoded_network(three_bodies, dev_ctx):
    """axs_mlp_predict = -D^{-1} v + decode(forward(features)) with the features
    (d, (2 kappa - (k_min + k_max)) / (k_max - k_min)), each step through its own
    library call; the wavenumbers given must be the context's."""
    from paper_1406_0236_amd import AxsError, FP64, Mlp, mlp_predict, warm_start_decode, warm_start_size
    wl, S = three_bodies
    ctx = _ctx(wl)
    mmax = 3
    P = warm_start_size(ctx, mmax)
    net, p, sizes, rng = _net(dev_ctx, 4, 32, 2, P, 13)
    dirs = wl.dirs
    kr = (1.5, 2.5)
    got = mlp_predict(net, ctx, dirs, kr, kappas=wl.kappa).cpu().numpy()
    feats = np.concatenate([dirs, np.full((len(dirs), 1), (2 * wl.kappa - sum(kr)) / (kr[1] - kr[0]))], axis=1)
    Yn = net.forward(torch.from_numpy(feats.astype(np.float32)).cuda())
    dec = warm_start_decode(ctx, Yn, dirs, mmax).cpu().numpy()
    v = ctx.incident_plane_waves(dirs)
    bt = -ctx.apply_precond(v, FP64).cpu().numpy()
    e = rel(got, bt + dec)
    print(f"predict vs -D^-1 v + decode(forward): {e:.2e}")
    assert e < 1e-12, e
    with pytest.raises(AxsError, match="EINVAL"):
        mlp_predict(net, ctx, dirs, kr, kappas=wl.kappa * 1.01)
    with pytest.raises(AxsError, match="EINVAL"):
        mlp_predict(net, ctx, dirs, (2.5, 1.5))
    wrong = Mlp(dev_ctx, 4, 8, 1, P + 2)
    with pytest.raises(AxsError, match="EINVAL"):
        mlp_predict(wrong, ctx, dirs, kr)
    wrong.close()
    net.close()
    ctx.close()


def test_learned_warm_start_against_single_body_guess():
    """Train on the mixed-body geometry (reduced: 12 wavenumbers x 32 directions),
    evaluate on held-out wavenumbers: the zero guess, the single-body responses
    b~ = -D^{-1} v (free: GMRES's first iterate lies in its span), and b~ plus the
    network's multiple-scattering part.  Every solve converges, and the learned
    guess has a smaller FP64 residual than b~ on average."""
    from paper_1406_0236_amd import Context, warm_start_size
    from paper_1406_0236_amd import warmstart as W
    from workloads import configs
    wl_at = lambda k: configs.mixed_bodies(kappa=k, disc_kappa=W.K_MAX, n_dirs=1)
    rng = np.random.default_rng(4)
    ks = rng.uniform(W.K_MIN, W.K_MAX, 12)
    dirs = [W.random_directions(32, rng) for _ in ks]
    X, Y = W.generate(wl_at, ks, dirs, mmax=8, tol=1e-8, log=print)
    dev = Context(0)
    ws = W.WarmStart(dev, Y.shape[1], width=256, depth=4)
    hist = ws.train(X, Y, epochs=150, batch=64, lr=1e-3, log=print)
    assert hist[-1] < 0.5 * hist[0]
    rng2 = np.random.default_rng(40)
    hk = rng2.uniform(W.K_MIN, W.K_MAX, 2)
    hd = [W.random_directions(16, rng2) for _ in hk]
    rows = W.evaluate(ws, wl_at, hk, hd, tol=1e-7, log=print)
    agg = W.summarise(rows)
    print(agg)
    assert all(a["converged"] for a in agg.values())
    assert agg["learned"]["guess_rel_residual"] < agg["single_body"]["guess_rel_residual"]
