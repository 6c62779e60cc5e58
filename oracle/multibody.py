"""Multibody Nystrom system and its solution, FP64 (reference).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3.3: the global matrix is the block matrix [A_pq] with diagonal blocks
from the single-body modal discretisation and off-diagonal blocks given by
the naive rule A(i, j) = G_kappa(x_i, x_j) w_j (eq. "nystromnaive"), because
the kernel is smooth between distinct bodies.
Sec. 4: A = D + B with D the block diagonal; GMRES is applied to
    sigma + D^{-1} B sigma = -D^{-1} v                       (eq. "precond").
The solution of that system is the solution of A sigma = -v (eq. "blocksystem").
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .modal import coupling
from .nystrom import Shape


class Body:
    def __init__(self, shape: Shape, centre, rot):
        self.shape = shape
        self.centre = np.asarray(centre, dtype=np.float64)
        self.rot = np.asarray(rot, dtype=np.float64)
        sh = shape
        th = 2.0 * math.pi * np.arange(sh.NF) / sh.NF
        ct, st = np.cos(th), np.sin(th)
        # node order within a body: contour node i major, azimuth l minor
        loc = np.stack([np.outer(sh.r, ct), np.outer(sh.r, st),
                        np.repeat(sh.z[:, None], sh.NF, axis=1)], axis=-1).reshape(-1, 3)
        nloc = np.stack([np.outer(sh.nr, ct), np.outer(sh.nr, st),
                         np.repeat(sh.nz[:, None], sh.NF, axis=1)], axis=-1).reshape(-1, 3)
        self.x = loc @ self.rot.T + self.centre
        self.n = nloc @ self.rot.T
        # surface weights (2 pi / N_F) r |gamma'| w_gauss (Sec. 3.2 tensor rule)
        self.w = np.repeat(sh.area_w * (2.0 * math.pi / sh.NF), sh.NF)
        self.size = sh.NG * sh.NF


class System:
    """All bodies of one problem (shared kappa and eta)."""

    def __init__(self, bodies):
        self.bodies = list(bodies)
        self.kappa = self.bodies[0].shape.kappa
        self.eta = self.bodies[0].shape.eta
        self.gamma = coupling(self.kappa, self.eta)
        for b in self.bodies:
            assert b.shape.kappa == self.kappa and b.shape.eta == self.eta
        self.offsets = np.cumsum([0] + [b.size for b in self.bodies])
        self.N = int(self.offsets[-1])
        self.x = np.concatenate([b.x for b in self.bodies])
        self.n = np.concatenate([b.n for b in self.bodies])
        self.w = np.concatenate([b.w for b in self.bodies])
        self.body_of = np.repeat(np.arange(len(self.bodies)), [b.size for b in self.bodies])

    @classmethod
    def from_workload(cls, wl, Nt=None):
        shapes = {}
        bodies = []
        for bs in wl.bodies:
            key = (id(bs.contour), bs.M)
            if key not in shapes:
                c = bs.contour
                shapes[key] = Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, wl.kappa, wl.eta, bs.M, Nt)
            bodies.append(Body(shapes[key], bs.centre, bs.rot))
        return cls(bodies)

    # -- kernel -------------------------------------------------------------
    def kernel(self, xt, xs, ns):
        """G_kappa(x_t, x_s) = d phi/d n(x_s) + gamma phi, phi = e^{i k R}/(4 pi R) (eq. Gkappa),
        gamma = i eta (kappa > 0) or eta (kappa = 0, the Laplace equation of Sec. 6.1)."""
        d = xt[:, None, :] - xs[None, :, :]
        R = np.sqrt(np.sum(d * d, axis=-1))
        nd = np.sum(ns[None, :, :] * d, axis=-1)
        k = self.kappa
        e = np.exp(1j * k * R) / (4.0 * math.pi * R)
        return e * (nd * (1.0 - 1j * k * R) / (R * R) + self.gamma)

    # -- operators on global vectors (N,) or (N, r) ------------------------------
    def apply_B(self, sigma, rows=None):
        """(B sigma)_i = sum_{j not in body(i)} G(x_i, x_j) w_j sigma_j (C/OpenMP sum)."""
        return apply_B_c(self, sigma, rows)

    def apply_B_numpy(self, sigma, rows=None, chunk=512):
        """The same sum as apply_B, in numpy (used to cross-check the C sum)."""
        sig = np.asarray(sigma, dtype=np.complex128)
        vec = sig.ndim == 1
        if vec:
            sig = sig[:, None]
        q = self.w[:, None] * sig
        rows = np.arange(self.N) if rows is None else np.asarray(rows)
        out = np.zeros((rows.size, sig.shape[1]), dtype=np.complex128)
        for a in range(0, rows.size, chunk):
            rr = rows[a:a + chunk]
            with np.errstate(divide="ignore", invalid="ignore"):
                G = self.kernel(self.x[rr], self.x, self.n)
            G[self.body_of[rr][:, None] == self.body_of[None, :]] = 0.0
            out[a:a + chunk] = G @ q
        return out[:, 0] if vec else out

    def _blockwise(self, fn, v):
        v = np.asarray(v, dtype=np.complex128)
        out = np.empty_like(v)
        for b, o0, o1 in zip(self.bodies, self.offsets[:-1], self.offsets[1:]):
            blk = v[o0:o1]
            sh = b.shape
            if blk.ndim == 1:
                out[o0:o1] = fn(sh, blk.reshape(sh.NG, sh.NF)).reshape(-1)
            else:
                r = blk.shape[1]
                x = np.moveaxis(blk.reshape(sh.NG, sh.NF, r), 2, 0)
                out[o0:o1] = np.moveaxis(fn(sh, x), 0, 2).reshape(-1, r)
        return out

    def apply_D(self, v):
        return self._blockwise(lambda sh, x: sh.apply_A(x), v)

    def apply_Dinv(self, v):
        return self._blockwise(lambda sh, x: sh.apply_Ainv(x), v)

    def apply_A(self, sigma):
        return self.apply_D(sigma) + self.apply_B(sigma)

    def matvec(self, sigma):
        """sigma + D^{-1} B sigma (eq. precond)."""
        return np.asarray(sigma) + self.apply_Dinv(self.apply_B(sigma))

    # -- right-hand sides -----------------------------------------------------
    def plane_waves(self, dirs):
        """v(x_i) = exp(i kappa d . x_i) for each direction: (N, r)."""
        d = np.atleast_2d(dirs)
        return np.exp(1j * self.kappa * (self.x @ d.T))

    def point_source_field(self, src, amp, x):
        """sum_s amp_s phi(x, x_s), phi = e^{ikR}/(4 pi R)."""
        d = x[:, None, :] - np.asarray(src)[None, :, :]
        R = np.sqrt(np.sum(d * d, axis=-1))
        return (np.exp(1j * self.kappa * R) / (4.0 * math.pi * R)) @ np.asarray(amp)

    def rhs(self, v):
        """b = -D^{-1} v."""
        return -self.apply_Dinv(v)

    # -- solutions ---------------------------------------------------------------
    def dense_matrix(self):
        """The full N x N Nystrom matrix A = D + B (small problems only)."""
        A = np.zeros((self.N, self.N), dtype=np.complex128)
        for b, o0, o1 in zip(self.bodies, self.offsets[:-1], self.offsets[1:]):
            A[o0:o1, o0:o1] = b.shape.dense_block()
        chunk = 512
        for a in range(0, self.N, chunk):
            rr = np.arange(a, min(self.N, a + chunk))
            with np.errstate(divide="ignore", invalid="ignore"):
                G = self.kernel(self.x[rr], self.x, self.n) * self.w[None, :]
            G[self.body_of[rr][:, None] == self.body_of[None, :]] = 0.0
            A[rr] += G
        return A

    def solve_dense(self, v):
        import scipy.linalg as sla
        return sla.solve(self.dense_matrix(), -np.asarray(v), overwrite_a=True)

    def eval_field(self, sigma, xt):
        """u(x) = sum_j G(x, x_j) w_j sigma_j (eq. intHelm1 with the surface rule)."""
        sig = np.asarray(sigma, dtype=np.complex128)
        q = self.w[:, None] * (sig[:, None] if sig.ndim == 1 else sig)
        out = np.zeros((len(xt), q.shape[1]), dtype=np.complex128)
        for a in range(0, self.N, 4096):
            G = self.kernel(np.asarray(xt), self.x[a:a + 4096], self.n[a:a + 4096])
            out += G @ q[a:a + 4096]
        return out[:, 0] if sig.ndim == 1 else out

    def far_field(self, sigma, xhat):
        """u_inf(xh) = (1/4pi) sum_j (-i k xh.n_j + i eta) e^{-i k xh.x_j} w_j sigma_j."""
        if not self.kappa > 0:
            raise ValueError("no far field at kappa = 0")
        xh = np.atleast_2d(xhat)
        sig = np.asarray(sigma, dtype=np.complex128)
        q = self.w[:, None] * (sig[:, None] if sig.ndim == 1 else sig)
        k = self.kappa
        E = np.exp(-1j * k * (xh @ self.x.T)) * (-1j * k * (xh @ self.n.T) + 1j * self.eta)
        out = (E @ q) / (4.0 * math.pi)
        return out[:, 0] if sig.ndim == 1 else out


def gmres(apply, b, tol=1e-12, max_iters=300, x0=None):
    """Plain GMRES (Saad-Schultz) with modified Gram-Schmidt and Givens rotations.

    Stops when ||b - A x|| / ||b|| <= tol.  Returns (x, iterations, residual history).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    r = b - apply(x) if x0 is not None else b.copy()
    bn = np.linalg.norm(b)
    beta = np.linalg.norm(r)
    hist = [beta / bn]
    if beta / bn <= tol:
        return x, 0, hist
    V = [r / beta]
    H = np.zeros((max_iters + 1, max_iters), dtype=np.complex128)
    cs = np.zeros(max_iters, dtype=np.complex128)
    sn = np.zeros(max_iters, dtype=np.complex128)
    g = np.zeros(max_iters + 1, dtype=np.complex128)
    g[0] = beta
    j = 0
    for j in range(max_iters):
        w = apply(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        # complex Givens rotation [[c, s], [-conj(s), c]], c real, zeroing H[j+1, j]
        a, bb = H[j, j], H[j + 1, j]
        den = math.hypot(abs(a), abs(bb))
        if abs(a) == 0.0:
            cs[j], sn[j] = 0.0, np.conj(bb) / abs(bb)
        else:
            cs[j], sn[j] = abs(a) / den, (a / abs(a)) * np.conj(bb) / den
        a0 = H[j, j]
        H[j, j] = cs[j] * a0 + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]) / bn)
        if hist[-1] <= tol:
            break
    k = j + 1
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = x + np.stack(V[:k], axis=1) @ y
    return x, k, hist


# ----------------------------------------------------------------------------
# large-N direct sum in C (same definition as System.apply_B, FP64, OpenMP)
# ----------------------------------------------------------------------------
_LIB = None


def _clib():
    global _LIB
    if _LIB is None:
        path = os.path.join(os.path.dirname(__file__), "c", "liboracle_direct.so")
        if not os.path.exists(path):
            from .build import build_c
            build_c()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_direct_rows.argtypes = [ctypes.c_int64, dp, dp, dp, lp, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int64, lp,
                                          ctypes.c_int64, dp]
        lib.oracle_direct_rows.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def apply_B_c(system: System, sigma, rows=None):
    """(B sigma) on the given rows via the C/OpenMP reference sum. sigma: (N,) or (N, r)."""
    lib = _clib()
    sig = np.asarray(sigma, dtype=np.complex128)
    vec = sig.ndim == 1
    if vec:
        sig = sig[:, None]
    r = sig.shape[1]
    q = np.ascontiguousarray((system.w[:, None] * sig).T)         # (r, N) complex
    x = np.ascontiguousarray(system.x)
    n = np.ascontiguousarray(system.n)
    body = np.ascontiguousarray(system.body_of.astype(np.int64))
    rows = np.arange(system.N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((r, rows.size), dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    rc = lib.oracle_direct_rows(system.N, x.ctypes.data_as(dp), n.ctypes.data_as(dp),
                                q.view(np.float64).ctypes.data_as(dp), body.ctypes.data_as(lp),
                                system.kappa, system.gamma.real, system.gamma.imag, r,
                                rows.ctypes.data_as(lp), rows.size,
                                out.view(np.float64).ctypes.data_as(dp))
    if rc != 0:
        raise RuntimeError("oracle_direct_rows failed")
    out = out.T
    return out[:, 0] if vec else out


def num_threads():
    return int(_clib().oracle_num_threads())
