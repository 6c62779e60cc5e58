"""Closed forms for a sound-soft sphere (used to pin the reference). TEST INFRASTRUCTURE ONLY.

  * Combined-field operator 1/2 I + D + i eta S on a sphere of radius a acts on
    the spherical harmonic Y_l^m with eigenvalue
        lambda_l = i kappa a^2 h_l(kappa a) [kappa j_l'(kappa a) + i eta j_l(kappa a)]
    (addition theorem for e^{ikR}/(4 pi R) and the jump relation of the double
    layer; h_l = h_l^(1)).
  * Mie series, plane wave exp(i kappa d.x), sound-soft sphere at the origin:
        u^s(x)   = -sum_l i^l (2l+1) [j_l(ka)/h_l(ka)] h_l(k|x|) P_l(d . x^)
        u_inf(x^) = (i/kappa) sum_l (2l+1) [j_l(ka)/h_l(ka)] P_l(d . x^)
    with u^s ~ e^{i kappa |x|}/|x| u_inf.
"""
import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def h1(l, x, derivative=False):
    return spherical_jn(l, x, derivative) + 1j * spherical_yn(l, x, derivative)


def sphere_eigenvalue(l, kappa, a, eta):
    ka = kappa * a
    return 1j * kappa * a * a * h1(l, ka) * (kappa * spherical_jn(l, ka, True)
                                             + 1j * eta * spherical_jn(l, ka))


def laplace_sphere_eigenvalue(l, a, eta):
    """Eigenvalue of 1/2 + K + eta S on Y_l for the sphere of radius a at kappa = 0, with
    S the single layer 1/(4 pi R) and K the double layer n(y).(x-y)/(4 pi R^3):
    S Y_l = a/(2l+1) Y_l (expansion of 1/|x-y| in Legendre polynomials with the
    addition theorem), and on the sphere n(y).(x-y) = -|x-y|^2/(2a), so K = -S/(2a):
    lambda_l = 1/2 - 1/(2(2l+1)) + eta a/(2l+1) = (l + eta a)/(2l+1)."""
    return (l + eta * a) / (2 * l + 1)


def mie_scattered(x, kappa, a, d, lmax=None):
    x = np.atleast_2d(x)
    rr = np.linalg.norm(x, axis=1)
    ct = (x @ np.asarray(d)) / rr
    ka = kappa * a
    lmax = lmax or int(ka + 30)
    u = np.zeros(len(x), dtype=np.complex128)
    for l in range(lmax + 1):
        u -= (1j ** l) * (2 * l + 1) * (spherical_jn(l, ka) / h1(l, ka)) * h1(l, kappa * rr) \
            * eval_legendre(l, ct)
    return u


def mie_far(xhat, kappa, a, d, lmax=None):
    xh = np.atleast_2d(xhat)
    ct = xh @ np.asarray(d)
    ka = kappa * a
    lmax = lmax or int(ka + 30)
    u = np.zeros(len(xh), dtype=np.complex128)
    for l in range(lmax + 1):
        u += (2 * l + 1) * (spherical_jn(l, ka) / h1(l, ka)) * eval_legendre(l, ct)
    return 1j / kappa * u
