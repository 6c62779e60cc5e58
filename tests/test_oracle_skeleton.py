"""Pins of the skeletonization reference (oracle/skeleton.py, Sec. 5), ring and
point versions, against what they must reproduce: the uncompressed solution,
the interpolation of fields of sources they never saw, the monotone growth of
the rank with accuracy, brute-force proxy fields, and the published output
sequence of the sketch's random generator.  CPU only."""
import numpy as np
import pytest

from oracle.multibody import System, gmres
from oracle.skeleton import SkeletonSystem, ring_id
from workloads import configs


@pytest.fixture(scope="module")
def two():
    wl = configs.two_spheres()
    S = System.from_workload(wl)
    return wl, S


def test_compressed_solve_reproduces_the_full_solution(two):
    """Eq. ip6 solved by GMRES and lifted back (eq. ip1) agrees with GMRES on the
    full preconditioned system to within the ID tolerance, in as many iterations,
    with fewer unknowns."""
    wl, S = two
    v = S.plane_waves(wl.dirs)[:, 0]
    x, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-12)
    K = SkeletonSystem(S, eps=1e-8)
    xs, its = K.solve(v, tol=1e-12)
    err = np.linalg.norm(xs - x) / np.linalg.norm(x)
    (k, NG, R_p), = K.ranks().values()
    print(f"rings {k} of {NG} (proxy radius {R_p:.2f}), unknowns {K.Ns} of {S.N}, "
          f"iterations {its} vs {it}, error {err:.2e}")
    assert k < 0.7 * NG and K.Ns == k * S.bodies[0].shape.NF * 2
    assert abs(its - it) <= 1
    assert err < 1e-8, err


def test_rank_grows_as_the_tolerance_tightens(two):
    wl, S = two
    sh = S.bodies[0].shape
    ks = [ring_id(sh, 2.0, eps)[1].shape[1] for eps in (1e-4, 1e-7, 1e-10)]
    print(f"ranks {ks}")
    assert ks[0] < ks[1] < ks[2] <= sh.NG


def _exterior_points(rng, n, r0, r1):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * rng.uniform(r0, r1, n)[:, None]


def test_skeleton_rings_interpolate_unseen_incoming_and_outgoing_fields(two):
    """The ID was built from combined-field sources on proxy spheres; here point
    sources at random places outside the proxy sphere (incoming) and random
    densities seen from random far targets (outgoing) must be reproduced from the
    skeleton rings alone, at every azimuthal node: u = (X (x) I) u(skeleton) and
    A_far sigma = A_far(:, skeleton) (X^T (x) I) sigma."""
    wl, S = two
    body = S.bodies[0]
    sh = body.shape
    eps = 1e-8
    I, X = ring_id(sh, 2.0, eps)
    NG, NF = sh.NG, sh.NF
    rng = np.random.default_rng(17)
    loc = body.x - body.centre
    # incoming: 12 point sources at radius 2.2 .. 4 around the body
    src = _exterior_points(rng, 12, 2.2, 4.0)
    d = loc[:, None, :] - src[None, :, :]
    R = np.linalg.norm(d, axis=-1)
    u = (np.exp(1j * S.kappa * R) / (4 * np.pi * R)) @ rng.standard_normal(12)
    U = u.reshape(NG, NF)
    e_in = np.linalg.norm(X @ U[I] - U) / np.linalg.norm(U)
    # outgoing: random density on the body, 20 targets at radius 2.2 .. 6
    tg = _exterior_points(rng, 20, 2.2, 6.0)
    sig = (rng.standard_normal(NG * NF) + 1j * rng.standard_normal(NG * NF))
    G = S.kernel(tg + body.centre, body.x, body.n) * S.w[:body.size][None, :]
    full = G @ sig
    sk = (np.sort(I)[:, None] * NF + np.arange(NF)[None, :]).ravel()
    Xs = X[:, np.argsort(I)]                                 # columns in sorted ring order
    red = G[:, sk] @ (Xs.T @ sig.reshape(NG, NF)).ravel()
    e_out = np.linalg.norm(red - full) / np.linalg.norm(full)
    print(f"k = {X.shape[1]}: incoming {e_in:.2e}, outgoing {e_out:.2e}")
    assert e_in < 1e-6 and e_out < 1e-6


# -- point skeletons (single-node index sets) ------------------------------------
from oracle.skeleton import (PointSkeletonSystem, gaussian_sketch, point_id, point_id_randomized,  # noqa: E402
                             point_matrix, proxy_rings, splitmix64)


@pytest.fixture(scope="module")
def two_small():
    """Two unit spheres 3 apart at kappa = pi, 6 x 8 Gauss nodes, |m| <= 12: N = 2,400."""
    wl = configs.two_spheres(n_panels=6, p=8, M=12)
    return wl, System.from_workload(wl)


def test_splitmix64_reproduces_the_published_sequence():
    """The generator's outputs from state 0 (state advanced by the golden-ratio
    increment before each output): the first three values of the reference
    implementation."""
    gamma = 0x9E3779B97F4A7C15
    states = np.array([0, gamma, (2 * gamma) % (1 << 64)], dtype=np.uint64)
    assert [int(v) for v in splitmix64(states)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_gaussian_sketch_is_standard_complex_normal_and_prefix_stable():
    om = gaussian_sketch(7, 200, 200)
    assert abs(om.mean()) < 0.03
    assert abs(np.mean(np.abs(om) ** 2) - 2.0) < 0.05
    assert abs(np.mean(om * om)) < 0.05                  # circular: E z^2 = 0
    assert np.array_equal(gaussian_sketch(7, 200, 50), om[:, :50])
    assert not np.allclose(gaussian_sketch(8, 200, 50), om[:, :50])


def _ring_points(r, z, nr, nz, Q):
    ph = 2.0 * np.pi * np.arange(Q) / Q
    x = np.stack([r * np.cos(ph), r * np.sin(ph), np.full(Q, z)], axis=1)
    n = np.stack([nr * np.cos(ph), nr * np.sin(ph), np.full(Q, nz)], axis=1)
    return ph, x, n


def test_point_matrix_columns_are_the_proxy_ring_fields(two_small):
    """Column (m, c) of the point proxy matrix against brute-force azimuthal sums
    of the 3-D kernel: the field at every node (i, l) of the proxy ring c of
    combined-field sources with density e^{i m phi} (incoming), and the
    coefficient of e^{i m phi} of each node's field along an outgoing proxy ring
    (column -m).  Each column is a real positive multiple of its brute-force
    field; a wrong sign of m or of theta_l, or a swapped node order, fails."""
    wl, S = two_small
    sh = S.bodies[0].shape
    NG, NF, M = sh.NG, sh.NF, sh.M
    R_p, npx, Q = 2.0, 12, 512
    H = point_matrix(sh, R_p, npx)
    Cp = 3 * npx
    th = 2.0 * np.pi * np.arange(NF) / NF
    x = np.stack([np.outer(sh.r, np.cos(th)), np.outer(sh.r, np.sin(th)),
                  np.repeat(sh.z[:, None], NF, axis=1)], axis=-1).reshape(-1, 3)
    nx = np.stack([np.outer(sh.nr, np.cos(th)), np.outer(sh.nr, np.sin(th)),
                   np.repeat(sh.nz[:, None], NF, axis=1)], axis=-1).reshape(-1, 3)
    pr, pz, pnr, pnz, pw = proxy_rings(R_p, npx)
    checked = 0
    for m in (3, -3, 0, 7):
        for c in (2, 9):
            ph, y, ny = _ring_points(pr[c], pz[c], pnr[c], pnz[c], Q)
            b = (S.kernel(x, y, ny) @ np.exp(1j * m * ph)) * (2 * np.pi / Q) * pw[c]
            h = H[:, (m + M) * Cp + c]
            a = np.vdot(h, b) / np.vdot(h, h)
            assert abs(a.imag) < 1e-10 * abs(a) and a.real > 0
            assert np.linalg.norm(b - a * h) < 1e-10 * np.linalg.norm(b), (m, c)
            checked += 1
        for c, R_o in ((4, R_p), (npx + 5, 1.25 * R_p)):
            qr, qz, _, _, qw = proxy_rings(R_o, npx)
            cc = c % npx
            ph, p, _ = _ring_points(qr[cc], qz[cc], 0.0, 0.0, Q)
            a_m = (S.kernel(p, x, nx).T @ np.exp(-1j * m * ph)) * (2 * np.pi / Q)
            b = a_m * np.repeat(sh.area_w, NF) * qw[cc]
            h = H[:, (-m + M) * Cp + npx + c]
            a = np.vdot(h, b) / np.vdot(h, h)
            assert abs(a.imag) < 1e-10 * abs(a) and a.real > 0
            assert np.linalg.norm(b - a * h) < 1e-10 * np.linalg.norm(b), (m, c)
            checked += 1
    assert checked == 16


@pytest.mark.parametrize("method", ["qrcp", "randomized"])
def test_point_id_interpolates_the_proxy_matrix(two_small, method):
    """X(I, :) is the identity and the other rows of H are X(J, :) H(I, :) to the
    ID tolerance; the randomized ID (sketch + QRCP of the sketch) keeps about as
    many nodes as the QRCP of H itself."""
    wl, S = two_small
    sh = S.bodies[0].shape
    eps, npx = 1e-8, 24
    H = point_matrix(sh, 2.0, npx)
    if method == "qrcp":
        I, X = point_id(sh, 2.0, eps, npx)
    else:
        I, X, ell = point_id_randomized(sh, 2.0, eps, npx, seed=3)
        kq = point_id(sh, 2.0, eps, npx)[0].size
        assert abs(I.size - kq) <= 0.1 * kq and ell >= I.size + 16
    assert len(set(I.tolist())) == I.size
    assert np.array_equal(X[I], np.eye(I.size))
    e = np.linalg.norm(H - X @ H[I]) / np.linalg.norm(H)
    print(f"{method}: k = {I.size} of {H.shape[0]}, interpolation error {e:.2e}")
    assert e < 10 * eps


@pytest.mark.parametrize("method", ["qrcp", "randomized"])
def test_point_skeleton_solve_reproduces_the_full_solution(two_small, method):
    """Eq. ip6 with single-node skeletons, solved and lifted back, agrees with
    the full preconditioned solve to within the ID tolerance in as many
    iterations, with fewer unknowns than the ring skeletons."""
    wl, S = two_small
    v = S.plane_waves(wl.dirs)[:, 0]
    x, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-12)
    K = PointSkeletonSystem(S, eps=1e-8, method=method, seed=5)
    xs, its = K.solve(v, tol=1e-12)
    err = np.linalg.norm(xs - x) / np.linalg.norm(x)
    ring = SkeletonSystem(S, eps=1e-8)
    print(f"{method}: unknowns {K.Ns} (rings {ring.Ns}) of {S.N}, iterations {its} vs {it}, error {err:.2e}")
    assert K.Ns < ring.Ns and abs(its - it) <= 1
    assert err < 1e-7, err


def test_point_skeleton_interpolates_unseen_fields(two_small):
    """Point sources outside the proxy sphere (incoming) and random densities
    seen from far targets (outgoing) are reproduced from the skeleton nodes:
    u = X u(I) and A_far sigma = A_far(:, I) X^T sigma."""
    wl, S = two_small
    body = S.bodies[0]
    sh = body.shape
    I, X, _ = point_id_randomized(sh, 2.0, 1e-8, seed=2)
    rng = np.random.default_rng(23)
    loc = body.x - body.centre
    src = _exterior_points(rng, 12, 2.2, 4.0)
    d = loc[:, None, :] - src[None, :, :]
    R = np.linalg.norm(d, axis=-1)
    u = (np.exp(1j * S.kappa * R) / (4 * np.pi * R)) @ rng.standard_normal(12)
    e_in = np.linalg.norm(X @ u[I] - u) / np.linalg.norm(u)
    tg = _exterior_points(rng, 20, 2.2, 6.0)
    n = sh.NG * sh.NF
    sig = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    G = S.kernel(tg + body.centre, body.x, body.n) * S.w[:n][None, :]
    full = G @ sig
    red = G[:, I] @ (X.T @ sig)
    e_out = np.linalg.norm(red - full) / np.linalg.norm(full)
    print(f"k = {I.size}: incoming {e_in:.2e}, outgoing {e_out:.2e}")
    assert e_in < 1e-6 and e_out < 1e-6


def test_zero_frequency_proxy_sees_every_degree():
    """At kappa = 0 the system's coupling is real (D + eta S); on a proxy sphere
    of radius R_p that layer has no interior field of degree l = eta R_p - 1
    (its factor is eta R_p - (l + 1)), so proxy sources with the system's
    coupling at eta = 1, R_p = 2 would miss every incoming dipole field.  The
    proxy sources carry i eta instead: the point ID of a sphere interpolates
    the fields of exterior point sources and of exterior dipoles."""
    from workloads import geometry as geo
    s = geo.sphere(1.0, 4, 10)
    bodies = [configs.BodySpec(s, np.array([0.0, 0.0, 0.0]), np.eye(3), 8),
              configs.BodySpec(s, np.array([5.0, 0.0, 0.0]), np.eye(3), 8)]
    S = System.from_workload(configs.Workload("laplace_pair", 0.0, 1.0, bodies, np.zeros((1, 3))))
    body = S.bodies[0]
    I, X = point_id(body.shape, 2.0, 1e-8)
    rng = np.random.default_rng(3)
    src = _exterior_points(rng, 12, 2.2, 4.0)
    d = (body.x - body.centre)[:, None, :] - src[None, :, :]
    R = np.linalg.norm(d, axis=-1)
    mono = (1.0 / (4 * np.pi * R)) @ rng.standard_normal(12)
    pdir = rng.standard_normal((12, 3))
    dip = (np.einsum("njc,jc->nj", d, pdir) / (4 * np.pi * R ** 3)) @ rng.standard_normal(12)
    for name, u in (("point sources", mono), ("dipoles", dip)):
        e = np.linalg.norm(X @ u[I] - u) / np.linalg.norm(u)
        print(f"kappa = 0, {name}: k = {I.size}, interpolation error {e:.2e}")
        assert e < 1e-7
