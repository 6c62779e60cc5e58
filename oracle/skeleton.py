"""Skeletonization of the inter-body blocks (Sec. 5), FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

Sec. 5 factors every off-diagonal block as A_pq = U_p A~_pq V_q^* + R_pq (eq.
ip0) with interpolative decompositions, so that A~_pq = A_pq(I_p, I_q) is a
submatrix of B, and replaces the preconditioned system by the smaller one
(eqs. ip3-ip6)

    s~ + S B~ s~ = -v~,   s~_p = V_p^* s_p,   v~_p = V_p^* A_pp^{-1} v_p,
    S_p = V_p^* A_pp^{-1} U_p,

whose factors come from a proxy surface that carries every field a body can
receive from, or send to, the others (Sec. 5, first item).

Reading (for bodies of revolution): the skeleton is a set of whole rings --
contour nodes with all their azimuthal nodes -- so U_p = X (x) I and
V_p^* = X^T (x) I with one NG x k matrix X per shape acting on the contour
index.  X is the row interpolative decomposition over the contour index of
the modal blocks, stacked over all modes m = 0..M,
    H = [ IN_m  |  OUT_m^T ]_m ,
IN_m: the field at the body's contour nodes of combined-field sources D + i eta S
on a proxy sphere of radius R_p (incoming; the coupling i eta at every
frequency, also at kappa = 0 where the system's own coupling is real), OUT_m: the field of the body's nodes
(weights included) at contour nodes of proxy spheres of radii R_p and 1.25 R_p
(outgoing); a ring that interpolates every mode interpolates every azimuthal
node.  The row ID comes from QR with column pivoting of H^*:
H^* P = Q R, rank k where |R_kk| < eps |R_00|, T = R_11^{-1} R_12,
H(J, :) = T^* H(I, :), so X(I, :) = Id and X(J, :) = T^*.  Then
A_pq ~ (X (x) I) A_pq(I_p, I_q) (X^T (x) I).

Point skeletons (Sec. 5 as printed, index sets of single nodes): the row ID
is over the N_G N_F nodes of the proxy matrix H[(i, l), (m, c)] = Hm[i, c]
e^{i m theta_l}, m = -M..M, so U_p = V_p = X (N_G N_F x k) and S_p = X^T
A_pp^{-1} X is a dense k x k matrix.  point_id is the QRCP of H^* (the
definition); point_id_randomized follows the remark of Sec. 5 on randomized
sampling: the QRCP of the Gaussian sketch (H Omega)^*, with Omega drawn by a
counter-based generator (SplitMix64 and the Box-Muller transform) so that the
library can draw the same sketch.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .modal import default_nt, modal_kernels
from .multibody import System, apply_B_c, gmres


def proxy_rings(R: float, n: int):
    """n Gauss-Legendre points in polar angle on the sphere of radius R:
    (r, z, n_r, n_z, w) with the outward normal and w = R^2 sin(theta) dtheta."""
    x, w = np.polynomial.legendre.leggauss(n)
    th = 0.5 * math.pi * (x + 1.0)
    wt = 0.5 * math.pi * w
    return (R * np.sin(th), R * np.cos(th), np.sin(th), np.cos(th), R * R * np.sin(th) * wt)


def modal_blocks(shape, R_p: float, n_in: int, n_out: int):
    """IN (M+1, NG, n_in) and OUT (M+1, 2 n_out, NG) of the docstring."""
    sh = shape
    Nt = default_nt(sh.kappa, 1.25 * R_p)     # band limit of the azimuthal integrands out to the proxy
    r_, z_, nr_, nz_, w_ = proxy_rings(R_p, n_in)
    # incoming: target body node i, source proxy node j (its normal, its weight)
    ti, sj = np.meshgrid(np.arange(sh.NG), np.arange(n_in), indexing="ij")
    ti, sj = ti.ravel(), sj.ravel()
    # the proxy's own sources carry the coupling i eta at every frequency: at
    # kappa = 0 the system's real coupling eta would make D + eta S blind to
    # the incoming fields of degree l with eta R_p = l + 1 (on a sphere of
    # radius R_p the interior field of that layer with density Y_l is
    # (eta R_p - (l + 1)) / (2l + 1) (r / R_p)^l Y_l)
    kS, kD, _ = modal_kernels(sh.r[ti], r_[sj], r_[sj] - sh.r[ti], z_[sj] - sh.z[ti], nr_[sj], nz_[sj],
                              sh.kappa, sh.eta, sh.M, Nt)
    kG = (kD + 1j * sh.eta * kS) / (4.0 * math.pi)
    IN = (kG.reshape(sh.NG, n_in, sh.M + 1) * w_[None, :, None]).transpose(2, 0, 1)
    outs = []
    for R_o in (R_p, 1.25 * R_p):
        r_o, z_o, _, _, w_o = proxy_rings(R_o, n_out)
        tj, si = np.meshgrid(np.arange(n_out), np.arange(sh.NG), indexing="ij")
        tj, si = tj.ravel(), si.ravel()
        _, _, kG = modal_kernels(r_o[tj], sh.r[si], sh.r[si] - r_o[tj], sh.z[si] - z_o[tj], sh.nr[si], sh.nz[si],
                                 sh.kappa, sh.eta, sh.M, Nt)
        outs.append(kG.reshape(n_out, sh.NG, sh.M + 1) * sh.area_w[None, :, None] * w_o[:, None, None])
    OUT = np.concatenate(outs, axis=0).transpose(2, 0, 1)
    return IN, OUT


def ring_id(shape, R_p: float, eps: float, n_in: int | None = None, n_out: int | None = None):
    """Skeleton rings I (pivot order) and the NG x k interpolation matrix X."""
    n_in = n_in or shape.NG
    n_out = n_out or shape.NG
    IN, OUT = modal_blocks(shape, R_p, n_in, n_out)
    IN = IN / np.linalg.norm(IN)
    OUT = OUT / np.linalg.norm(OUT)
    H = np.concatenate([np.concatenate([IN[m], OUT[m].T], axis=1) for m in range(shape.M + 1)], axis=1)
    _, R, piv = sla.qr(H.conj().T, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    k = int(np.sum(d > eps * d[0]))
    I, J = piv[:k], piv[k:]
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])
    X = np.zeros((shape.NG, k), dtype=np.complex128)
    X[I, :] = np.eye(k)
    X[J, :] = T.conj().T
    return I, X


def proxy_radius(system: System, b: int, factor: float = 2.0) -> float:
    """The largest sphere around body b's centre that stays out of every other
    body's bounding ball, capped at factor x its own bounding radius."""
    body = system.bodies[b]
    rb = np.max(np.linalg.norm(body.x - body.centre, axis=1))
    gap = min(np.linalg.norm(body.centre - o.centre) - np.max(np.linalg.norm(o.x - o.centre, axis=1))
              for q, o in enumerate(system.bodies) if q != b)
    return min(factor * rb, gap), rb


class _Nodes:
    """A node subset in the form the C reference sum takes (x, n, w, body_of)."""

    def __init__(self, x, n, w, body_of, kappa, gamma):
        self.x, self.n, self.w, self.body_of = x, n, w, body_of
        self.N = len(w)
        self.kappa, self.gamma = kappa, gamma


class SkeletonSystem:
    """The compressed system of eq. ip6 for a System, one ring ID per shape.

    A shape whose proxy sphere would not clear its own bounding ball (R_p <
    1.05 r_b) keeps all its rings (X = Id)."""

    def __init__(self, system: System, eps: float = 1e-10, factor: float = 2.0):
        self.S = system
        self.eps = eps
        shapes = {}
        for b, body in enumerate(system.bodies):
            R_p, rb = proxy_radius(system, b, factor)
            key = id(body.shape)
            shapes.setdefault(key, [body.shape, R_p, rb])
            shapes[key][1] = min(shapes[key][1], R_p)
        self.ids = {}
        for key, (sh, R_p, rb) in shapes.items():
            if R_p < 1.05 * rb:
                self.ids[key] = (np.arange(sh.NG), np.eye(sh.NG, dtype=np.complex128), R_p)
            else:
                I, X = ring_id(sh, R_p, eps)
                self.ids[key] = (I, X, R_p)
        # skeleton nodes: the rings I of every body, all azimuthal nodes, in body order
        idx, self.sk_off = [], [0]
        for body, o0 in zip(system.bodies, system.offsets[:-1]):
            I = self.ids[id(body.shape)][0]
            rings = np.sort(I)
            nodes = (o0 + rings[:, None] * body.shape.NF + np.arange(body.shape.NF)[None, :]).ravel()
            idx.append(nodes)
            self.sk_off.append(self.sk_off[-1] + nodes.size)
        self.sk = np.concatenate(idx)
        self.nodes = _Nodes(system.x[self.sk], system.n[self.sk], system.w[self.sk], system.body_of[self.sk],
                            system.kappa, system.gamma)
        self.Ns = self.sk.size

    def ranks(self):
        return {key: (X.shape[1], X.shape[0], R_p) for key, (I, X, R_p) in self.ids.items()}

    def _X(self, body):
        """X with its rows ordered like the sorted skeleton rings (the node order)."""
        I, X, _ = self.ids[id(body.shape)]
        order = np.argsort(I)
        return X[:, order]

    # -- the factors of eq. ip3 applied body by body --------------------------------
    def U(self, ws):
        """U_p w on every body: skeleton values (Ns, r) -> all nodes (N, r)."""
        out = np.zeros((self.S.N,) + ws.shape[1:], dtype=np.complex128)
        for body, o0, o1, s0, s1 in zip(self.S.bodies, self.S.offsets[:-1], self.S.offsets[1:],
                                        self.sk_off[:-1], self.sk_off[1:]):
            X = self._X(body)
            blk = ws[s0:s1].reshape(X.shape[1], body.shape.NF, -1)
            out[o0:o1] = np.einsum("ik,klr->ilr", X, blk).reshape(o1 - o0, -1).reshape(out[o0:o1].shape)
        return out

    def Vstar(self, w):
        """V_p^* w on every body: all nodes (N, r) -> skeleton (Ns, r), V^* = X^T (x) I."""
        out = np.zeros((self.Ns,) + w.shape[1:], dtype=np.complex128)
        for body, o0, o1, s0, s1 in zip(self.S.bodies, self.S.offsets[:-1], self.S.offsets[1:],
                                        self.sk_off[:-1], self.sk_off[1:]):
            X = self._X(body)
            blk = w[o0:o1].reshape(body.shape.NG, body.shape.NF, -1)
            out[s0:s1] = np.einsum("ik,ilr->klr", X, blk).reshape(s1 - s0, -1).reshape(out[s0:s1].shape)
        return out

    def apply_Btilde(self, sig_s):
        """A~_pq summed: the inter-body sum over skeleton nodes only (a submatrix of B)."""
        return apply_B_c(self.nodes, sig_s)

    def apply_S(self, ws):
        """S_p = V_p^* A_pp^{-1} U_p on every body."""
        return self.Vstar(self.S.apply_Dinv(self.U(ws)))

    def matvec(self, sig_s):
        """s~ + S B~ s~ (eq. ip6)."""
        return sig_s + self.apply_S(self.apply_Btilde(sig_s))

    def rhs(self, v):
        """-v~ = -V^* A^{-1} v."""
        return -self.Vstar(self.S.apply_Dinv(v))

    def recover(self, sig_s, v):
        """s_p = -A_pp^{-1} (v_p + U_p sum_q A~_pq s~_q)  (eq. ip1 with the factorisation)."""
        return -self.S.apply_Dinv(v + self.U(self.apply_Btilde(sig_s)))

    def solve(self, v, tol=1e-12, max_iters=300):
        """GMRES on eq. ip6, then the full density; returns (sigma, iterations)."""
        xs, it, _ = gmres(self.matvec, self.rhs(v), tol=tol, max_iters=max_iters)
        return self.recover(xs, v), it


# ---------------------------------------------------------------------------
# Point skeletons (Sec. 5 as printed: the index sets I_p are single nodes).
# ---------------------------------------------------------------------------
def default_n_proxy(kappa: float, R_p: float) -> int:
    """Polar Gauss points per proxy sphere for the point version: the fields on a
    sphere of radius 1.25 R_p have polar band limit about kappa 1.25 R_p, plus a
    margin of 40 for the decay to the ID tolerance (40 at kappa = 0)."""
    return 40 + int(math.ceil(1.25 * kappa * R_p))


def point_matrix(shape, R_p: float, n_proxy: int):
    """The proxy matrix of one body at the level of its nodes (body frame).

    Rows: the N_G N_F nodes (i, l) in node order i N_F + l.  Columns: (m, c) for
    m = -M..M (outer) and the proxy columns c of the ring version (inner: n_proxy
    incoming, then 2 n_proxy outgoing), column index (m + M) C' + c,

        H[(i, l), (m, c)] = Hm[i, c] e^{i m theta_l},  Hm = [IN_|m| | OUT_|m|^T],

    IN and OUT each scaled to unit Frobenius norm over m = 0..M as in ring_id.
    A proxy ring of combined-field sources with the azimuthal profile
    e^{i m phi} produces at node (i, l) the field IN_m[i, c] e^{i m theta_l} (the
    kernel depends on theta - phi only, and k_{-m} = k_m); a node's field at a
    proxy ring, expanded in the proxy azimuth, has the coefficient of e^{i m phi}
    equal to OUT_m[c, i] e^{-i m theta_l}, which is column (-m, c) of the same
    matrix.  So the columns span both the incoming and the outgoing fields of
    Sec. 5 (first item) at every node."""
    IN, OUT = modal_blocks(shape, R_p, n_proxy, n_proxy)
    IN = IN / np.linalg.norm(IN)
    OUT = OUT / np.linalg.norm(OUT)
    NG, NF, M = shape.NG, shape.NF, shape.M
    th = 2.0 * math.pi * np.arange(NF) / NF
    cols = []
    for m in range(-M, M + 1):
        Hm = np.concatenate([IN[abs(m)], OUT[abs(m)].T], axis=1)          # (NG, C')
        cols.append((Hm[:, None, :] * np.exp(1j * m * th)[None, :, None]).reshape(NG * NF, -1))
    return np.concatenate(cols, axis=1)


def _id_from_rows(n, piv_rows, T):
    """X (n x k) with X(I, :) = Id and X(J, :) = T for I = piv_rows[:k] (pivot
    order), J = piv_rows[k:]."""
    k = T.shape[1]
    X = np.zeros((n, k), dtype=np.complex128)
    X[piv_rows[:k], :] = np.eye(k)
    X[piv_rows[k:], :] = T
    return X


def point_id(shape, R_p: float, eps: float, n_proxy: int | None = None):
    """Deterministic row ID of point_matrix (the definition): QR with column
    pivoting of H^*, rank k where |R_kk| < eps |R_00|, X(J, :) = (R_11^{-1} R_12)^*.
    Returns the skeleton nodes I (pivot order) and X (N_G N_F x k)."""
    n_proxy = n_proxy or default_n_proxy(shape.kappa, R_p)
    H = point_matrix(shape, R_p, n_proxy)
    _, R, piv = sla.qr(H.conj().T, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    k = int(np.sum(d > eps * d[0]))
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])
    return piv[:k], _id_from_rows(H.shape[0], piv, T.conj().T)


# -- the counter-based Gaussian draws of the randomized ID ---------------------------
_MASK64 = (1 << 64) - 1


def splitmix64(x):
    """Steele, Lea and Flood's SplitMix64 output function of the state x (the
    state advanced by the golden-ratio increment 0x9E3779B97F4A7C15, then two
    xor-shift-multiply rounds and a final xor-shift); numpy uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def uniform01(seed: int, k):
    """Uniform draw k of stream `seed` in (0, 1): the top 53 bits of
    splitmix64(seed * 0x632BE59BD9B4E019 + k), centred in their interval."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = np.uint64((seed * 0x632BE59BD9B4E019) & _MASK64) + k
    return ((splitmix64(x) >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def gaussian_sketch(seed: int, rows: int, cols: int):
    """Omega (rows x cols) complex Gaussian, entry (r, s) from draw e = s rows + r
    (so the first columns do not depend on cols) by the Box-Muller transform:
    sqrt(-2 ln u1) e^{2 pi i u2}, u1 = uniform01(seed, 2e), u2 = uniform01(seed, 2e + 1)."""
    e = (np.arange(cols, dtype=np.uint64)[None, :] * np.uint64(rows) + np.arange(rows, dtype=np.uint64)[:, None])
    u1 = uniform01(seed, 2 * e)
    u2 = uniform01(seed, 2 * e + 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.exp(2j * math.pi * u2)


def point_id_randomized(shape, R_p: float, eps: float, n_proxy: int | None = None, seed: int = 1,
                        ell0: int = 256, oversample: int = 16):
    """Randomized row ID of point_matrix (Sec. 5, remark on randomized
    sampling): the sketch Y = H Omega (n x ell, Omega complex Gaussian) has,
    with high probability, the row structure of H, so rows that interpolate Y
    interpolate H.  The rows come from QR with column pivoting of Y^*, rank k
    where |R_kk| < eps |R_00|, X(J, :) = (R_11^{-1} R_12)^* as in point_id.  The
    sketch width ell doubles from ell0 (capped by the sizes of H) until
    k <= ell - oversample.  Returns (I in pivot order, X, ell)."""
    n_proxy = n_proxy or default_n_proxy(shape.kappa, R_p)
    H = point_matrix(shape, R_p, n_proxy)
    n, C = H.shape
    cap = min(n, C)
    ell = min(ell0, cap)
    while True:
        Y = H @ gaussian_sketch(seed, C, ell)
        _, R, piv = sla.qr(Y.conj().T, mode="economic", pivoting=True)
        d = np.abs(np.diag(R))
        k = int(np.sum(d > eps * d[0]))
        if k <= ell - oversample or ell == cap:
            break
        ell = min(2 * ell, cap)
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])
    return piv[:k], _id_from_rows(n, piv, T.conj().T), ell


class PointSkeletonSystem(SkeletonSystem):
    """The compressed system of eq. ip6 with single-node skeletons: U_p = V_p = X
    (N_G N_F x k, body node order), S_p = X^T A_pp^{-1} X dense, B~ the inter-body
    sum over the skeleton nodes.  method: "qrcp" (point_id) or "randomized"
    (point_id_randomized with the given seed)."""

    def __init__(self, system: System, eps: float = 1e-8, factor: float = 2.0, n_proxy: int | None = None,
                 method: str = "qrcp", seed: int = 1):
        self.S = system
        self.eps = eps
        shapes = {}
        for b, body in enumerate(system.bodies):
            R_p, rb = proxy_radius(system, b, factor)
            key = id(body.shape)
            shapes.setdefault(key, [body.shape, R_p, rb])
            shapes[key][1] = min(shapes[key][1], R_p)
        self.ids = {}
        for key, (sh, R_p, rb) in shapes.items():
            n = sh.NG * sh.NF
            if R_p < 1.05 * rb:
                self.ids[key] = (np.arange(n), np.eye(n, dtype=np.complex128), R_p)
            elif method == "qrcp":
                I, X = point_id(sh, R_p, eps, n_proxy)
                self.ids[key] = (I, X, R_p)
            else:
                I, X, _ = point_id_randomized(sh, R_p, eps, n_proxy, seed)
                self.ids[key] = (I, X, R_p)
        idx, self.sk_off = [], [0]
        for body, o0 in zip(system.bodies, system.offsets[:-1]):
            nodes = o0 + np.sort(self.ids[id(body.shape)][0])
            idx.append(nodes)
            self.sk_off.append(self.sk_off[-1] + nodes.size)
        self.sk = np.concatenate(idx)
        self.nodes = _Nodes(system.x[self.sk], system.n[self.sk], system.w[self.sk], system.body_of[self.sk],
                            system.kappa, system.gamma)
        self.Ns = self.sk.size

    def U(self, ws):
        """X w on every body: skeleton values (Ns, r) -> all nodes (N, r)."""
        out = np.zeros((self.S.N,) + ws.shape[1:], dtype=np.complex128)
        for body, o0, o1, s0, s1 in zip(self.S.bodies, self.S.offsets[:-1], self.S.offsets[1:],
                                        self.sk_off[:-1], self.sk_off[1:]):
            out[o0:o1] = np.tensordot(self._X(body), ws[s0:s1], axes=(1, 0))
        return out

    def Vstar(self, w):
        """X^T w on every body: all nodes (N, r) -> skeleton (Ns, r)."""
        out = np.zeros((self.Ns,) + w.shape[1:], dtype=np.complex128)
        for body, o0, o1, s0, s1 in zip(self.S.bodies, self.S.offsets[:-1], self.S.offsets[1:],
                                        self.sk_off[:-1], self.sk_off[1:]):
            out[s0:s1] = np.tensordot(self._X(body).T, w[o0:o1], axes=(1, 0))
        return out
