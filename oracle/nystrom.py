"""Single-body Nystrom discretisation in Fourier space, FP64 (reference).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 3.2: the surface rule is the tensor product of a composite
Gauss-Legendre rule on the generating curve and the trapezoidal rule in the
azimuth; the BIE decouples into one equation per Fourier mode m on the curve,

    1/2 sigma_m(y) + int_gamma k^G_m(y, y') sigma_m(y') r' |gamma'| ds' = -v_m(y),

whose discretisation is the block-diagonal matrix A~ of eq. (A = F* A~ F).
Entries of mode m (the paper leaves the singular rule to a cited
Kolm-Rokhlin table; here an equivalent product-integration reading):

  * far panel:  K_m(i, j) = k^G_m(y_i, y_j) r_j |gamma'_j| w_j   (naive Nystrom entry)
  * near panel (the target's own panel, its neighbours along the curve, and
    any panel closer to y_i than that panel's arc length):
        K_m(i, j) = int_{-1}^{1} k^G_m(y_i, y(s)) l_j(s) r(s) |gamma'(s)| ds
    with l_j the Lagrange basis on the panel's Gauss nodes and y(s), gamma'(s)
    the degree-(p-1) interpolants of the node data.  The integral is taken by
    tanh-sinh quadrature split at the target parameter (or nearest node),
    refined until two successive step sizes agree.

  A~_m = 1/2 I + K_m;  S_m = A~_m^{-1} by LU (scipy).  A~_{-m} = A~_m.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .modal import default_nt, modal_kernels


def gl_nodes(p):
    return np.polynomial.legendre.leggauss(p)


def lagrange_matrix(nodes, s):
    """L[k, j] = l_j(s_k) for the Lagrange basis on `nodes` (plain product form)."""
    s = np.asarray(s, dtype=np.float64)
    p = nodes.size
    L = np.ones((s.size, p))
    for j in range(p):
        for k in range(p):
            if k != j:
                L[:, j] *= (s - nodes[k]) / (nodes[j] - nodes[k])
    return L


def lagrange_deriv_matrix(nodes, s):
    """D[k, j] = l_j'(s_k), by the product rule (no division by s - s_j)."""
    s = np.asarray(s, dtype=np.float64)
    p = nodes.size
    D = np.zeros((s.size, p))
    for j in range(p):
        for m in range(p):
            if m == j:
                continue
            term = np.full(s.size, 1.0 / (nodes[j] - nodes[m]))
            for k in range(p):
                if k != j and k != m:
                    term *= (s - nodes[k]) / (nodes[j] - nodes[k])
            D[:, j] += term
    return D


class Shape:
    """One generating contour with its wavenumber, coupling and mode cutoff."""

    def __init__(self, rz, drz, gw, n_panels, p, kappa, eta, M, Nt=None):
        self.rz = np.asarray(rz, dtype=np.float64)
        self.drz = np.asarray(drz, dtype=np.float64)
        self.gw = np.asarray(gw, dtype=np.float64)
        self.n_panels, self.p = int(n_panels), int(p)
        self.NG = self.n_panels * self.p
        assert self.rz.shape == (self.NG, 2)
        self.kappa, self.eta, self.M = float(kappa), float(eta), int(M)
        self.NF = 2 * self.M + 1
        self.r, self.z = self.rz[:, 0], self.rz[:, 1]
        self.dr, self.dz = self.drz[:, 0], self.drz[:, 1]
        self.speed = np.hypot(self.dr, self.dz)
        self.nr = -self.dz / self.speed      # outward normal (-z', r')/|gamma'|
        self.nz = self.dr / self.speed
        self.area_w = self.r * self.speed * self.gw      # weight of int_gamma f r dl
        self.s_nodes, _ = gl_nodes(self.p)
        self.panel_len = (self.speed * self.gw).reshape(self.n_panels, self.p).sum(axis=1)
        rmax = max(float(np.max(self.r)), 1e-3)
        self.Nt = Nt or default_nt(self.kappa, rmax)
        self._At = None
        self._S = None

    # -- geometry on a panel -------------------------------------------------
    def panel_interp(self, P, s):
        """Position interpolant on panel P at parameters s: (r, z, L)."""
        L = lagrange_matrix(self.s_nodes, s)
        sl = slice(P * self.p, (P + 1) * self.p)
        return L @ self.r[sl], L @ self.z[sl], L

    def panel_curve(self, i, P, s):
        """Source data on near panel P for target node i at parameters s.

        The curve on a near panel is the degree-(p-1) interpolant of the node
        positions; its derivative gives the normal and the line element, so
        that n'.(y' - y) vanishes to second order as y' -> y.  On the target's
        own panel the displacement is sum_{k != i} (y_k - y_i) l_k(s), which is
        accurate to rounding relative to |s - s_i|.
        Returns (rp, dr, dz, nr, nz, speed, L).
        """
        sl = slice(P * self.p, (P + 1) * self.p)
        L = lagrange_matrix(self.s_nodes, s)
        D = lagrange_deriv_matrix(self.s_nodes, s)
        rp = L @ self.r[sl]
        rs, zs = D @ self.r[sl], D @ self.z[sl]
        if P == i // self.p:
            dr = L @ (self.r[sl] - self.r[i])
            dz = L @ (self.z[sl] - self.z[i])
        else:
            dr = rp - self.r[i]
            dz = L @ self.z[sl] - self.z[i]
        sp = np.hypot(rs, zs)
        return rp, dr, dz, -zs / sp, rs / sp, sp, L

    def near_panels(self, i):
        """Panels treated by product integration for target node i."""
        own = i // self.p
        near = []
        ends = [-1.0, 1.0]
        for P in range(self.n_panels):
            if abs(P - own) <= 1:
                near.append(P)
                continue
            sl = slice(P * self.p, (P + 1) * self.p)
            d = np.hypot(self.r[sl] - self.r[i], self.z[sl] - self.z[i])
            re, ze, _ = self.panel_interp(P, ends)
            de = np.hypot(re - self.r[i], ze - self.z[i])
            if min(d.min(), de.min()) < self.panel_len[P]:
                near.append(P)
        return near

    def split_point(self, i, P):
        """Parameter on panel P where the integrand for target i is (nearly) singular."""
        own = i // self.p
        if P == own:
            return float(self.s_nodes[i % self.p])
        cand = np.concatenate([[-1.0], self.s_nodes, [1.0]])
        re, ze, _ = self.panel_interp(P, cand)
        k = int(np.argmin(np.hypot(re - self.r[i], ze - self.z[i])))
        return float(cand[k])

    # -- product integration ---------------------------------------------------
    @staticmethod
    def _tanh_sinh(a, b, h, tmax=4.0):
        """Nodes, weights and the distances to both ends for int_a^b by tanh-sinh."""
        tau = np.arange(-tmax, tmax + 0.5 * h, h)
        u = 0.5 * math.pi * np.sinh(tau)
        da = (b - a) / (1.0 + np.exp(-2.0 * u))          # x - a
        db = (b - a) / (1.0 + np.exp(2.0 * u))           # b - x
        x = np.where(da < db, a + da, b - db)
        w = h * 0.5 * (b - a) * 0.5 * math.pi * np.cosh(tau) / np.cosh(u) ** 2
        # nodes closer to an end than 1e-15 of the interval are dropped: what they
        # would add to an integrand with a log end singularity is below 1e-13
        keep = (np.minimum(da, db) > 1e-15 * (b - a)) & (w > 0)
        return x[keep], w[keep]

    def _integrand(self, i, P, s):
        rp, dr, dz, nr, nz, sp, L = self.panel_curve(i, P, s)
        # points on the symmetry axis (r -> 0 at a pole) carry zero area weight
        ok = (rp > 1e-13) & (np.hypot(dr, dz) > 0)
        _, _, kG = modal_kernels(self.r[i], rp[ok], dr[ok], dz[ok], nr[ok], nz[ok],
                                 self.kappa, self.eta, self.M, self.Nt)
        return kG, L[ok], rp[ok] * sp[ok], ok

    def product_integral(self, i, P, h=1.0 / 16, check=True):
        """(M+1, p) entries K_m(i, j) for the p nodes j of near panel P."""
        sp = self.split_point(i, P)
        pieces = [(a, b) for a, b in ((-1.0, sp), (sp, 1.0)) if b - a > 1e-14]

        def run(hh):
            tot = np.zeros((self.M + 1, self.p), dtype=np.complex128)
            for a, b in pieces:
                x, w = self._tanh_sinh(a, b, hh)
                kG, L, jac, ok = self._integrand(i, P, x)
                tot += np.einsum("km,k,kj->mj", kG, w[ok] * jac, L)
            return tot

        val = run(h)
        if check:
            # refine until two successive step sizes agree to 5e-13 of the largest
            # entry: the rule converges double-exponentially, so the finer value's
            # quadrature error is far below that difference, which then is the
            # integrand's own rounding.  The differences level off at that
            # rounding floor (1.6e-13 to 8e-13 seen); at the finest step a
            # difference up to 2e-12 is taken as the floor.
            prev = run(2 * h)
            hh = h
            while True:
                scale = max(np.max(np.abs(val)), 1e-300)
                err = np.max(np.abs(val - prev)) / scale
                if err <= 5e-13:
                    break
                if hh < h / 32:
                    if err <= 2e-12:
                        break
                    raise RuntimeError(f"product integral not converged: {err}")
                hh *= 0.5
                prev, val = val, run(hh)
        return val

    # -- modal matrices ----------------------------------------------------------
    def modal_row(self, i, check=True):
        """K_m(i, :) for all m: array (M+1, NG)."""
        row = np.zeros((self.M + 1, self.NG), dtype=np.complex128)
        near = self.near_panels(i)
        mask = np.ones(self.NG, dtype=bool)
        for P in near:
            mask[P * self.p:(P + 1) * self.p] = False
        far = np.nonzero(mask)[0]
        if far.size:
            _, _, kG = modal_kernels(self.r[i], self.r[far], self.r[far] - self.r[i],
                                     self.z[far] - self.z[i], self.nr[far], self.nz[far],
                                     self.kappa, self.eta, self.M, self.Nt)
            row[:, far] = (kG * self.area_w[far][:, None]).T
        for P in near:
            row[:, P * self.p:(P + 1) * self.p] = self.product_integral(i, P, check=check)
        return row

    def modal_matrices(self, check=True):
        """A~_m = 1/2 I + K_m for m = 0..M: array (M+1, NG, NG)."""
        if self._At is None:
            K = np.zeros((self.M + 1, self.NG, self.NG), dtype=np.complex128)
            for i in range(self.NG):
                K[:, i, :] = self.modal_row(i, check=check)
            K += 0.5 * np.eye(self.NG)[None]
            self._At = K
        return self._At

    def inverses(self):
        """S_m = A~_m^{-1} by LU with partial pivoting (per mode)."""
        if self._S is None:
            At = self.modal_matrices()
            S = np.empty_like(At)
            I = np.eye(self.NG, dtype=np.complex128)
            for m in range(self.M + 1):
                lu = sla.lu_factor(At[m])
                S[m] = sla.lu_solve(lu, I)
            self._S = S
        return self._S

    # -- body-local operators on nodal vectors (NG, NF) ------------------------
    def mode_index(self):
        """|m| for each FFT bin k = 0..NF-1 (m = k for k <= M, k - NF otherwise)."""
        k = np.arange(self.NF)
        return np.where(k <= self.M, k, self.NF - k)

    def apply_modal(self, mats, sigma):
        """F^{-1} diag(mats_|m|) F applied to sigma of shape (..., NG, NF)."""
        X = np.fft.fft(sigma, axis=-1)
        Y = np.empty_like(X)
        am = self.mode_index()
        for k in range(self.NF):
            Y[..., :, k] = np.einsum("ij,...j->...i", mats[am[k]], X[..., :, k])
        return np.fft.ifft(Y, axis=-1)

    def apply_A(self, sigma):
        return self.apply_modal(self.modal_matrices(), sigma)

    def apply_Ainv(self, sigma):
        return self.apply_modal(self.inverses(), sigma)

    def dense_block(self):
        """The nodal diagonal block A_bb (n x n, node order (i, l)) = F^{-1} A~ F."""
        At = self.modal_matrices()
        am = self.mode_index()
        # circulant in l - l': c[i, j, d] = (1/NF) sum_k A~_{|m_k|}[i, j] e^{2 pi i k d / NF}
        T = At[am]                                   # (NF, NG, NG) indexed by bin k
        c = np.fft.ifft(T, axis=0)                   # (NF: d, NG, NG)
        n = self.NG * self.NF
        D = np.empty((self.NG, self.NF, self.NG, self.NF), dtype=np.complex128)
        l = np.arange(self.NF)
        dmat = (l[:, None] - l[None, :]) % self.NF
        for i in range(self.NG):
            D[i] = np.transpose(c[dmat][:, :, i, :], (0, 2, 1))
        return D.reshape(n, n)
