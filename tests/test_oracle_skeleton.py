"""Pins of the ring skeletonization reference (oracle/skeleton.py, Sec. 5) against
what it must reproduce: the uncompressed solution, the interpolation of fields
of sources it never saw, and the monotone growth of the rank with accuracy.
CPU only."""
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
