"""Azimuthal Fourier modes of the combined-field kernel, FP64 (reference).

TEST INFRASTRUCTURE ONLY: the oracle is imported by tests, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.

Sec. 3.2 decouples the BIE on a body of revolution into one equation per
Fourier mode (eqs. for the Fourier series of v, sigma and G_kappa and the
sequence of BIEs on the generating curve).  Its modal kernels ("toroidal
harmonics") are computed by a method the paper only cites; here they are the
exact Fourier integrals, evaluated in closed form as follows.

With t = theta - theta', chi = (r^2 + r'^2 + (z - z')^2) / (2 r r') and
R(t)^2 = 2 r r' (chi - cos t):

  k^S_m = int_0^{2pi} e^{-imt} e^{i kappa R}/R dt
        = sum_l c_l q_{m-l} + i s_m,
    c_l : Fourier coefficients of cos(kappa R(t))   (entire in R^2, so exact by FFT)
    s_m : modes of sin(kappa R)/R                   (entire in R^2, exact by FFT)
    q_m = int e^{-imt}/R dt = 2 Q_{|m|-1/2}(chi) / sqrt(r r'),
          Q = Legendre function of the second kind (toroidal harmonic).

  k^D_m = n_r' d/dr' k^S_m + n_z' d/dz' k^S_m  (normal derivative at the source)
  k^G_m = (k^D_m + gamma k^S_m) / (4 pi)       (eq. for G_kappa, 1/(4pi) from phi)

with the single-layer coupling gamma = i eta for kappa > 0 (Sec. 2) and
gamma = eta at kappa = 0, where the paper's Laplace equation (Sec. 6.1) adds
the single layer with a real coefficient (eta = 1 there).

All modes are even in m because G depends on t only through cos t.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipe, ellipkm1


def toroidal_q(chi: np.ndarray, chim1: np.ndarray, nmax: int):
    """Q_{mu-1/2}(chi) and dQ_{mu-1/2}/dchi for mu = 0..nmax.

    chi > 1; chim1 = chi - 1 supplied separately to keep precision as chi -> 1.
    Q_{-1/2} = sqrt(2/(chi+1)) K(2/(chi+1)) and Q_{1/2} = chi Q_{-1/2}
    - sqrt(2 (chi+1)) E(2/(chi+1)) (K, E with parameter m = k^2); higher
    orders from (nu+1) Q_{nu+1} = (2nu+1) chi Q_nu - nu Q_{nu-1}.  The forward
    recurrence loses about exp(2 mu eta) relative accuracy (chi = cosh eta), so
    it is used only while 2 nmax eta <= 2; otherwise the ratio
    Q_{nu+1}/Q_nu is obtained by the backward (Miller) continued fraction and
    multiplied up from Q_{-1/2}.
    Returns (Q, dQ) of shape chi.shape + (nmax+1,).
    """
    chi = np.asarray(chi, dtype=np.float64)
    chim1 = np.asarray(chim1, dtype=np.float64)
    shp = chi.shape
    chi = chi.ravel()
    chim1 = chim1.ravel()
    P = chi.size
    Q = np.zeros((P, nmax + 2))          # index mu -> Q_{mu-1/2}; extra slot for Q_{nmax+1/2}
    p = chim1 / (chi + 1.0)              # 1 - m, m = 2/(chi+1)
    kk = np.sqrt(2.0 / (chi + 1.0))
    Kp = ellipkm1(p)
    Ep = ellipe(1.0 - p)
    q0 = kk * Kp
    Q[:, 0] = q0
    eta = np.arccosh(np.maximum(chi, 1.0))
    # eta computed stably for chi close to 1
    small = chim1 < 1e-3
    eta[small] = 2.0 * np.arcsinh(np.sqrt(0.5 * chim1[small]))
    fwd = 2.0 * (nmax + 1) * eta <= 2.0
    if np.any(fwd):
        i = np.nonzero(fwd)[0]
        x = chi[i]
        qa = q0[i]
        qb = x * kk[i] * Kp[i] - np.sqrt(2.0 * (x + 1.0)) * Ep[i]
        Q[i, 1] = qb
        for mu in range(1, nmax + 1):
            # nu = mu - 1/2:  (nu+1) Q_{nu+1} = (2nu+1) chi Q_nu - nu Q_{nu-1}
            qc = (2.0 * mu * x * qb - (mu - 0.5) * qa) / (mu + 0.5)
            Q[i, mu + 1] = qc
            qa, qb = qb, qc
    if np.any(~fwd):
        i = np.nonzero(~fwd)[0]
        x = chi[i]
        et = eta[i]
        extra = int(math.ceil(20.0 / float(np.min(et)))) + 20
        top = nmax + 1 + extra
        rho = 1.0 / (x + np.sqrt((x - 1.0) * (x + 1.0)))    # limit ratio e^{-eta}
        ratios = np.empty((i.size, nmax + 1))
        for mu in range(top, 0, -1):
            # rho_mu = Q_{mu+1/2}/Q_{mu-1/2};  rho_{mu-1} = (mu-1/2)/(2 mu chi - (mu+1/2) rho_mu)
            rho = (mu - 0.5) / (2.0 * mu * x - (mu + 0.5) * rho)
            if mu - 1 <= nmax:
                ratios[:, mu - 1] = rho
        qa = q0[i]
        for mu in range(0, nmax + 1):
            qa = qa * ratios[:, mu]
            Q[i, mu + 1] = qa
    # derivative: Q'_nu = nu (chi Q_nu - Q_{nu-1}) / (chi^2 - 1), with Q_{-3/2} = Q_{1/2}
    c2m1 = (chim1 * (chi + 1.0))[:, None]
    mu = np.arange(nmax + 1)[None, :]
    nu = mu - 0.5
    Qm1 = np.concatenate([Q[:, 1:2], Q[:, 0:nmax]], axis=1)
    dQ = nu * (chi[:, None] * Q[:, :nmax + 1] - Qm1) / c2m1
    return Q[:, :nmax + 1].reshape(shp + (nmax + 1,)), dQ.reshape(shp + (nmax + 1,))


def _tcos_series(x):
    """(x cos x - sin x)/x^3 by its Taylor series sum_{k>=1} (-1)^k 2k x^{2k-2}/(2k+1)!."""
    out = np.zeros_like(x)
    term_fact = 1.0
    for k in range(1, 12):
        term_fact = math.factorial(2 * k + 1)
        out = out + ((-1) ** k) * (2 * k) * x ** (2 * k - 2) / term_fact
    return out


def default_nt(kappa: float, r_max: float) -> int:
    """Samples in t: the kernel factors are band-limited to about kappa (r + r')."""
    need = 2.0 * kappa * 2.0 * r_max + 64.0
    nt = 32
    while nt < need:
        nt *= 2
    return nt


def coupling(kappa: float, eta: float) -> complex:
    """Coefficient of the single layer in G: i eta (Helmholtz, Sec. 2), eta at kappa = 0
    (the Laplace equation of Sec. 6.1)."""
    return 1j * eta if kappa > 0 else complex(eta)


def modal_kernels(r, rp, dr, dz, nrp, nzp, kappa: float, eta: float, M: int, Nt: int):
    """k^S_m, k^D_m, k^G_m for m = 0..M; arrays broadcast to a common shape P.

    Target at radius r; source at radius rp with unit normal (nrp, nzp) in the
    (r, z) half-plane; (dr, dz) = (rp - r, zp - z) is the source-minus-target
    displacement in that half-plane, passed in so that callers can form it
    without cancellation for sources next to the target.
    Returns complex arrays of shape (P, M+1).
    """
    r, rp, dr, dz, nrp, nzp = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64).ravel()
                                                    for a in (r, rp, dr, dz, nrp, nzp)))
    L = Nt // 2 - 1
    t = 2.0 * math.pi * np.arange(Nt) / Nt
    s2 = np.sin(0.5 * t)[None, :] ** 2
    d0sq = dr * dr + dz * dz
    ndel = nrp * dr + nzp * dz                                # n' . (y' - y)
    R2 = d0sq[:, None] + 4.0 * (r * rp)[:, None] * s2
    R = np.sqrt(R2)
    kR = kappa * R
    C = np.cos(kR)
    Sd = kappa * np.sinc(kR / math.pi)                       # sin(kR)/R
    with np.errstate(divide="ignore", invalid="ignore"):
        T = np.where(kR > 0.2, (kR * np.cos(kR) - np.sin(kR)) / np.where(R > 0, R ** 3, 1.0),
                     kappa ** 3 * _tcos_series(kR))
    # g(t) = n' . d/2 grad' R^2 = nrp (rp - r cos t) + nzp (zp - z)
    g = ndel[:, None] + 2.0 * (nrp * r)[:, None] * s2
    c = np.fft.rfft(C, axis=1).real / Nt                      # c_l, l = 0..Nt/2
    dc = np.fft.rfft(-kappa * Sd * g, axis=1).real / Nt       # n . grad' of c_l
    s = np.fft.rfft(Sd, axis=1).real * (2.0 * math.pi / Nt)   # s_m
    ds = np.fft.rfft(T * g, axis=1).real * (2.0 * math.pi / Nt)
    nmax = M + L
    chim1 = d0sq / (2.0 * r * rp)
    chi = 1.0 + chim1
    Qv, dQv = toroidal_q(chi, chim1, nmax)
    srr = np.sqrt(r * rp)[:, None]
    q = 2.0 * Qv / srr
    # n' . grad' chi = (n'.d)/(r rp) - nrp |d|^2 / (2 r rp^2)
    ndchi = (ndel / (r * rp) - nrp * d0sq / (2.0 * r * rp * rp))[:, None]
    dq = 2.0 * dQv * ndchi / srr - (nrp / (2.0 * rp))[:, None] * q
    # convolution over l in [-L, L]:  sum_l c_|l| q_|m-l|
    ls = np.arange(-L, L + 1)
    ms = np.arange(M + 1)
    idx = np.abs(ms[:, None] - ls[None, :])                   # (M+1, 2L+1)
    cl = c[:, np.abs(ls)]                                     # (P, 2L+1)
    dcl = dc[:, np.abs(ls)]
    qi = q[:, idx]                                            # (P, M+1, 2L+1)
    dqi = dq[:, idx]
    kS = np.einsum("pl,pml->pm", cl, qi) + 1j * s[:, :M + 1]
    kD = (np.einsum("pl,pml->pm", dcl, qi) + np.einsum("pl,pml->pm", cl, dqi)
          + 1j * ds[:, :M + 1])
    kG = (kD + coupling(kappa, eta) * kS) / (4.0 * math.pi)
    return kS, kD, kG
