"""Pins of the FP64 reference implementation against closed forms, independent
libraries (mpmath, scipy) and physical invariants.  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import lpmv

from oracle import analytic
from oracle.modal import modal_kernels, toroidal_q
from oracle.multibody import System, apply_B_c, gmres
from oracle.nystrom import Shape
from workloads import configs, geometry as geo


# --------------------------------------------------------------------------
# toroidal harmonics and modal kernels (Sec. 3.2)
# --------------------------------------------------------------------------

def test_toroidal_q_matches_mpmath_legenq():
    mp.mp.dps = 30
    chis = np.array([1.0 + 1e-9, 1.0 + 3e-5, 1.002, 1.05, 1.7, 4.0, 40.0])
    nmax = 60
    Q, dQ = toroidal_q(chis, chis - 1.0, nmax)
    for a, chi in enumerate(chis):
        for mu in (0, 1, 2, 7, 23, 60):
            ref = float(mp.re(mp.legenq(mu - 0.5, 0, mp.mpf(chi), type=3)))
            assert abs(Q[a, mu] - ref) <= 1e-12 * abs(ref) + 1e-300, (chi, mu)
            # derivative by a central difference of the mpmath function
            h = mp.mpf(chi - 1) * mp.mpf("1e-8")
            dref = float(mp.re((mp.legenq(mu - 0.5, 0, chi + h, type=3)
                                - mp.legenq(mu - 0.5, 0, chi - h, type=3)) / (2 * h)))
            assert abs(dQ[a, mu] - dref) <= 1e-7 * abs(dref) + 1e-300, (chi, mu)


def _brute_mode(r, z, rp, zp, nrp, nzp, k, eta, m):
    """int_0^{2pi} e^{-imt} G(t) dt straight from the kernel definition (mpmath)."""
    mp.mp.dps = 30

    def G(t):
        R = mp.sqrt((r - rp) ** 2 + (z - zp) ** 2 + 4 * r * rp * mp.sin(t / 2) ** 2)
        ph = mp.exp(1j * k * R) / R
        nd = nrp * (r * mp.cos(t) - rp) + nzp * (z - zp)       # n' . (x - x')
        return mp.exp(-1j * m * t) * (nd * (1 - 1j * k * R) / R ** 2 * ph + 1j * eta * ph) / (4 * mp.pi)
    eps = [mp.mpf(10) ** (-e) for e in (1, 2, 3, 4, 5, 6)]
    pts = [0] + eps[::-1] + [mp.pi] + [2 * mp.pi - e for e in eps] + [2 * mp.pi]
    return complex(mp.quad(G, pts))


@pytest.mark.parametrize("case", [
    (0.7, 0.2, 0.5, -0.3, 0.6, 0.8),          # generic
    (0.9, 0.1, 0.9001, 0.1002, 0.8, 0.6),     # nearly coincident, off-curve normal
    (0.3, 0.9, 0.05, 0.99, 0.1, 0.995),       # source next to the axis
    (1.2, -0.4, 0.2, 0.8, -0.7, 0.7),         # far apart
])
def test_modal_kernel_matches_bruteforce_quadrature(case):
    r, z, rp, zp, nr, nz = case
    nn = math.hypot(nr, nz)
    nr, nz = nr / nn, nz / nn
    k, M = 4 * math.pi, 12
    _, _, kG = modal_kernels(r, rp, rp - r, zp - z, nr, nz, k, k, M, 128)
    scale = np.max(np.abs(kG))
    for m in (0, 1, 5, 12):
        ref = _brute_mode(r, z, rp, zp, nr, nz, k, k, m)
        assert abs(kG[0, m] - ref) <= 1e-11 * scale, (case, m, kG[0, m], ref)


def test_modal_kernels_resum_to_kernel():
    """sum_m k_m e^{imt} / (2 pi) reproduces G(t) for a separated pair (normalisation)."""
    r, z, rp, zp, nr, nz = 0.8, 0.3, 0.5, -0.6, 0.6, -0.8
    k, M = 3.0, 60
    _, _, kG = modal_kernels(r, rp, rp - r, zp - z, nr, nz, k, 0.7, M, 128)
    t = 0.9
    m = np.arange(-M, M + 1)
    val = np.sum(kG[0, np.abs(m)] * np.exp(1j * m * t)) / (2 * math.pi)
    x = np.array([r, 0.0, z])
    y = np.array([rp * math.cos(-t), rp * math.sin(-t), zp])   # theta - theta' = t
    ny = np.array([nr * math.cos(-t), nr * math.sin(-t), nz])
    d = x - y
    R = np.linalg.norm(d)
    G = np.exp(1j * k * R) / (4 * math.pi * R) * (ny @ d * (1 - 1j * k * R) / R ** 2 + 1j * 0.7)
    assert abs(val - G) <= 1e-12 * abs(G)


# --------------------------------------------------------------------------
# quadrature and geometry (Sec. 3.2, tensor-product rule)
# --------------------------------------------------------------------------

def _system_of(contour, M, k=1.0):
    wl = configs.Workload("q", k, k, [configs.BodySpec(contour, np.zeros(3), np.eye(3), M)],
                          np.array([[0, 0, 1.0]]))
    return System.from_workload(wl)


def test_quadrature_sphere_and_spheroid_area_volume():
    S = _system_of(geo.sphere(1.3, 8, 10), 10)
    assert abs(S.w.sum() - 4 * math.pi * 1.3 ** 2) < 1e-12
    # divergence theorem: (1/3) int n . x dA = volume; positive only for outward n
    assert abs(np.sum(S.w * np.sum(S.n * S.x, axis=1)) / 3 - 4 / 3 * math.pi * 1.3 ** 3) < 1e-12
    a, c = 1.0, 2.5
    S = _system_of(geo.prolate(a, c, 16, 10), 10)
    e = math.sqrt(1 - a * a / (c * c))
    area = 2 * math.pi * a * a * (1 + c / (a * e) * math.asin(e))
    assert abs(S.w.sum() - area) < 1e-10 * area
    assert abs(np.sum(S.w * np.sum(S.n * S.x, axis=1)) / 3 - 4 / 3 * math.pi * a * a * c) < 1e-10


def test_quadrature_bowl_normal_outward_and_area():
    b = geo.bowl(6, 3, 6, 10)
    S = _system_of(b, 12)
    R, th, al = 1.0, 0.2, 2 * math.pi / 3
    ri, rc = R - th, th / 2
    # area: two spherical caps + the rim (half a torus tube about the circle of radius rm sin(al))
    caps = 2 * math.pi * (R * R + ri * ri) * (1 - math.cos(al))
    rm = R - rc
    # rim: surface of revolution of a half circle of radius rc centred at rho0 = rm sin al,
    # Pappus: length pi rc times 2 pi times centroid distance from the axis
    rho0 = rm * math.sin(al)
    # centroid of the half circle bulging along e_alpha = (cos al, sin al): offset 2 rc / pi
    cen_r = rho0 + (2 * rc / math.pi) * math.cos(al)
    rim = math.pi * rc * 2 * math.pi * cen_r
    assert abs(S.w.sum() - (caps + rim)) < 1e-9 * (caps + rim)
    assert np.sum(S.w * np.sum(S.n * S.x, axis=1)) > 0


# --------------------------------------------------------------------------
# modal Nystrom matrices: sphere eigenvalues (closed form)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sphere_shape():
    c = geo.sphere(1.0, 10, 10)
    k = math.pi
    return Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, k, k, 20), c


def test_sphere_modal_matrices_have_closed_form_eigenvalues(sphere_shape):
    sh, c = sphere_shape
    At = sh.modal_matrices()
    x = c.rz[:, 1]
    worst, worst_low = 0.0, 0.0
    for m in (0, 1, 2, 5, 9):
        for l in range(m, 11):
            lam = analytic.sphere_eigenvalue(l, sh.kappa, 1.0, sh.eta)
            v = lpmv(m, l, x)
            err = np.max(np.abs(At[m] @ v - lam * v)) / np.max(np.abs(lam * v))
            worst = max(worst, err)
            if l <= 5:
                worst_low = max(worst_low, err)
    # 100 contour nodes: seen 2e-10 at l = 10 (resolution), 1e-13 for l <= 5
    assert worst < 1e-9, worst
    assert worst_low < 1e-12, worst_low


def test_sphere_eigenvalue_pin_detects_wrong_sign_of_coupling(sphere_shape):
    """The same pin fails for the other sign of the single-layer coupling."""
    sh, c = sphere_shape
    At = sh.modal_matrices()
    v = lpmv(0, 3, c.rz[:, 1])
    lam_wrong = analytic.sphere_eigenvalue(3, sh.kappa, 1.0, -sh.eta)
    assert np.max(np.abs(At[0] @ v - lam_wrong * v)) > 1e-2


@pytest.fixture(scope="module")
def laplace_sphere_shape():
    c = geo.sphere(1.0, 10, 10)
    return Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, 0.0, 1.0, 20), c


def test_laplace_sphere_modal_matrices_have_closed_form_eigenvalues(laplace_sphere_shape):
    """kappa = 0, eta = 1 (Sec. 6.1): 1/2 + K + S has eigenvalues (l + 1)/(2l + 1) on the
    unit sphere; the same pin with eta = -1 must fail."""
    sh, c = laplace_sphere_shape
    At = sh.modal_matrices()
    x = c.rz[:, 1]
    worst, worst_low = 0.0, 0.0
    for m in (0, 1, 2, 5, 9):
        for l in range(m, 11):
            lam = analytic.laplace_sphere_eigenvalue(l, 1.0, sh.eta)
            v = lpmv(m, l, x)
            err = np.max(np.abs(At[m] @ v - lam * v)) / np.max(np.abs(lam * v))
            worst = max(worst, err)
            if l <= 5:
                worst_low = max(worst_low, err)
    assert worst < 1e-9, worst
    assert worst_low < 1e-12, worst_low
    v = lpmv(0, 3, x)
    assert np.max(np.abs(At[0] @ v - analytic.laplace_sphere_eigenvalue(3, 1.0, -1.0) * v)) > 1e-2


def test_modal_inverse_is_inverse(sphere_shape):
    sh, _ = sphere_shape
    S = sh.inverses()
    At = sh.modal_matrices()
    for m in (0, 7, 20):
        assert np.max(np.abs(S[m] @ At[m] - np.eye(sh.NG))) < 1e-12


# --------------------------------------------------------------------------
# single body: Mie series (textbook special case of -D^{-1} v)
# --------------------------------------------------------------------------

def test_single_sphere_matches_mie_series():
    wl = configs.single_sphere()
    S = System.from_workload(wl)
    d = np.array([0.0, 0.0, 1.0])
    v = S.plane_waves(d)[:, 0]
    sigma = S.rhs(v)                 # single body: sigma = -D^{-1} v exactly
    rng = np.random.default_rng(1)
    xt = geo.sphere_targets(10, 3.0, np.zeros(3), rng)
    u = S.eval_field(sigma, xt)
    ref = analytic.mie_scattered(xt, S.kappa, 1.0, d)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    assert err < 1e-8, err
    xh = geo.uniform_directions(8, rng)
    uf = S.far_field(sigma, xh)
    reff = analytic.mie_far(xh, S.kappa, 1.0, d)
    assert np.max(np.abs(uf - reff)) / np.max(np.abs(reff)) < 1e-8


# --------------------------------------------------------------------------
# inter-body operator and multibody solves (Secs. 3.3, 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["helmholtz", "laplace"])
def test_interbody_sum_rows_match_mpmath(which, small_system, laplace_system):
    wl, S = small_system if which == "helmholtz" else laplace_system
    rng = np.random.default_rng(3)
    sig = rng.standard_normal(S.N) + 1j * rng.standard_normal(S.N)
    rows = np.array([0, 17, S.N - 1, S.offsets[1] + 5])
    out = apply_B_c(S, sig, rows)
    mp.mp.dps = 30
    k, eta = S.kappa, S.eta
    gam = 1j * eta if k > 0 else eta          # single-layer coupling (Secs. 2 and 6.1)
    for a, i in enumerate(rows):
        acc = mp.mpc(0)
        for j in range(S.N):
            if S.body_of[j] == S.body_of[i]:
                continue
            d = [mp.mpf(S.x[i, c]) - mp.mpf(S.x[j, c]) for c in range(3)]
            R = mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            nd = sum(mp.mpf(S.n[j, c]) * d[c] for c in range(3))
            phi = mp.exp(1j * k * R) / (4 * mp.pi * R)
            acc += phi * (nd * (1 - 1j * k * R) / R ** 2 + gam) * mp.mpf(S.w[j]) * mp.mpc(sig[j])
        ref = complex(acc)
        assert abs(out[a] - ref) <= 1e-13 * max(abs(ref), 1e-3), (i, out[a], ref)


@pytest.mark.parametrize("which", ["helmholtz", "laplace"])
def test_c_sum_matches_numpy_sum(which, small_system, laplace_system):
    wl, S = small_system if which == "helmholtz" else laplace_system
    rng = np.random.default_rng(4)
    sig = rng.standard_normal((S.N, 3)) + 1j * rng.standard_normal((S.N, 3))
    a = apply_B_c(S, sig)
    b = S.apply_B_numpy(sig)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_gmres_solves_a_known_system():
    rng = np.random.default_rng(5)
    n = 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres(lambda v: A @ v, b, tol=1e-13)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
    assert hist[-1] <= 1e-13 and it <= n


def test_preconditioned_gmres_matches_dense_solve(small_system):
    wl, S = small_system
    v = S.plane_waves(wl.dirs)[:, 0]
    x, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-13)
    xd = S.solve_dense(v)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_greens_identity_point_sources(small_system):
    """Interior point sources: the exterior field is known exactly (Sec. 6 protocol)."""
    wl, S = small_system
    src = configs.point_sources(wl, seed=11)
    amp = np.ones(len(src))
    v = S.point_source_field(src, amp, S.x)
    x, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-12)
    xt = configs.exterior_targets(wl, 10, seed=12)
    u = S.eval_field(x, xt)
    ref = -S.point_source_field(src, amp, xt)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    assert err < 1e-6, err


def test_laplace_greens_identity_point_sources(laplace_system):
    """kappa = 0: interior point sources 1/(4 pi R) give the exterior field exactly
    (the accuracy protocol of Sec. 6 for the Laplace examples).  Sources sit in the
    sphere and the spheroid; the bowl's thin wall (0.2) would need panels of its own
    scale for a source inside it, so it only scatters."""
    wl, S = laplace_system
    src = configs.point_sources(wl, seed=13)
    amp = np.array([1.0, -0.7, 0.0])
    v = S.point_source_field(src, amp, S.x)
    x, it, _ = gmres(S.matvec, S.rhs(v), tol=1e-12)
    xt = configs.exterior_targets(wl, 10, seed=14)
    u = S.eval_field(x, xt)
    ref = -S.point_source_field(src, amp, xt)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print(f"Laplace Green's identity: {it} iterations, rel err {err:.2e}")
    assert err < 1e-6, err
    assert np.isrealobj(S.kernel(S.x[:2], S.x[-2:], S.n[-2:])) is False   # complex dtype kept
    assert np.max(np.abs(S.kernel(S.x[:2], S.x[-2:], S.n[-2:]).imag)) == 0.0  # but real at kappa = 0


def test_bowl_thin_wall_greens_identity_helmholtz():
    """kappa = 2 pi (the bowl 2 wavelengths across): two point sources inside the
    bowl's 0.2-thick wall, 0.1 from both faces, so the boundary data are nearly
    singular across the wall and every panel of the opposite face is a near
    panel of the product integration (Sec. 3.2).  A single body is solved
    exactly by its modal inverses, and its exterior field must equal minus the
    sources' field (the Sec. 6 protocol).  200 contour nodes (panels about the
    wall's thickness) and |m| <= 60 (the data's azimuthal content: 1.1e-3 at
    |m| <= 20, 2.5e-5 at 40, 8.7e-8 at 60, the same at 290 contour nodes)."""
    k = 2.0 * math.pi
    bw = geo.bowl(8, 2, 10, 10)
    wl = configs.Workload("bowl_wall", k, k, [configs.BodySpec(bw, np.zeros(3), np.eye(3), 60)], np.zeros((1, 3)))
    S = System.from_workload(wl)
    rng = np.random.default_rng(31)
    src = np.array([geo.interior_point(bw, rng) for _ in range(2)])
    for y in src:   # mid-wall: 0.1 from the inner (radius 0.8) and outer (radius 1) faces
        assert abs(np.linalg.norm(y) - 0.9) < 1e-12
    amp = np.array([1.0, -0.6 + 0.3j])
    sigma = S.rhs(S.point_source_field(src, amp, S.x))
    xt = geo.sphere_targets(10, 3.0, np.zeros(3), rng)
    u = S.eval_field(sigma, xt)
    ref = -S.point_source_field(src, amp, xt)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print(f"bowl wall, kappa = 2 pi: E_inf {err:.2e}")
    assert err < 1e-6, err


def test_reciprocity_and_optical_theorem(small_system):
    wl, S = small_system
    d1 = np.array([0.0, 0.6, 0.8])
    d2 = np.array([0.48, -0.6, 0.64])
    v = S.plane_waves(np.stack([d1, -d2]))
    sol = np.stack([gmres(S.matvec, S.rhs(v[:, c]), tol=1e-12)[0] for c in range(2)], axis=1)
    u12 = S.far_field(sol[:, 0], d2)       # u_inf(x^ = d2; d = d1)
    u21 = S.far_field(sol[:, 1], -d1)      # u_inf(x^ = -d1; d = -d2)
    assert abs(u12 - u21) <= 1e-6 * abs(u12), (u12, u21)
    # optical theorem (4 pi / k) Im u_inf(d; d) = int_{S^2} |u_inf|^2
    nth, nph = 40, 80
    xg, wg = np.polynomial.legendre.leggauss(nth)
    ph = 2 * math.pi * np.arange(nph) / nph
    st = np.sqrt(1 - xg * xg)
    dirs = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                     np.repeat(xg, nph)], axis=1)
    wq = np.repeat(wg, nph) * 2 * math.pi / nph
    uf = S.far_field(sol[:, 0], dirs)
    lhs = 4 * math.pi / S.kappa * S.far_field(sol[:, 0], d1).imag
    rhs = np.sum(wq * np.abs(uf) ** 2)
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
