"""Planted mistakes in the FP64 reference (on the CPU, in the reference only):
each plausible slip -- the sign of the coupling, a dropped double layer, a
transposed matrix, flipped normals, a lost radius in the weights, the wrong
jump term -- must make the closed-form sphere pin fail, while the reference as
written passes it.  This shows that the pins of tests/test_oracle_pins.py
would catch such slips.  A small sphere (4 panels x 10 nodes, modes 0-3,
kappa = eta = pi) keeps each rebuild to a second or two."""
import math

import numpy as np
import pytest
from scipy.special import lpmv

import oracle.modal as omodal
import oracle.nystrom as onys
from oracle import analytic
from workloads import geometry as geo


def _sphere():
    c = geo.sphere(1.0, 4, 10)
    return onys.Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, math.pi, math.pi, 3), c


def _pin_error(At, sh, c):
    """Largest relative violation of A~_m P_l^m = lambda_l P_l^m, m <= l <= 5."""
    x = c.rz[:, 1]
    worst = 0.0
    for m in range(4):
        for l in range(m, 6):
            lam = analytic.sphere_eigenvalue(l, sh.kappa, 1.0, sh.eta)
            v = lpmv(m, l, x)
            worst = max(worst, np.max(np.abs(At[m] @ v - lam * v)) / np.max(np.abs(lam * v)))
    return worst


def test_reference_as_written_passes():
    sh, c = _sphere()
    e = _pin_error(sh.modal_matrices(), sh, c)
    print(f"unmutated: {e:.2e}")
    assert e < 1e-8


def test_wrong_coupling_sign_fails(monkeypatch):
    orig = omodal.coupling
    monkeypatch.setattr(omodal, "coupling", lambda kappa, eta: -orig(kappa, eta))
    sh, c = _sphere()
    assert _pin_error(sh.modal_matrices(), sh, c) > 1e-3


def test_dropped_double_layer_fails(monkeypatch):
    orig = onys.modal_kernels

    def single_layer_only(*a, **k):
        kS, kD, kG = orig(*a, **k)
        return kS, kD, kG - kD / (4 * math.pi)
    monkeypatch.setattr(onys, "modal_kernels", single_layer_only)
    sh, c = _sphere()
    assert _pin_error(sh.modal_matrices(), sh, c) > 1e-3


def test_transposed_modal_matrices_fail():
    sh, c = _sphere()
    At = np.transpose(sh.modal_matrices(), (0, 2, 1))
    assert _pin_error(At, sh, c) > 1e-3


def test_flipped_normals_fail():
    sh, c = _sphere()
    sh.nr, sh.nz = -sh.nr, -sh.nz
    assert _pin_error(sh.modal_matrices(), sh, c) > 1e-3


def test_weights_without_the_radius_fail():
    sh, c = _sphere()
    sh.area_w = sh.area_w / sh.r
    assert _pin_error(sh.modal_matrices(), sh, c) > 1e-3


@pytest.mark.parametrize("jump", [-0.5, 0.0, 1.0])
def test_wrong_jump_term_fails(jump):
    sh, c = _sphere()
    At = sh.modal_matrices() + (jump - 0.5) * np.eye(sh.NG)[None]
    assert _pin_error(At, sh, c) > 1e-3


# --------------------------------------------------------------------------
# the inter-body operator B: Green's identity (interior point sources, exact
# exterior field) on the two-body system must break for a slip in B
# --------------------------------------------------------------------------

def _greens_error(S, wl):
    from oracle.multibody import gmres
    from workloads import configs
    src = configs.point_sources(wl, seed=11)
    amp = np.ones(len(src))
    v = S.point_source_field(src, amp, S.x)
    x, _, _ = gmres(S.matvec, S.rhs(v), tol=1e-10, max_iters=100)
    xt = configs.exterior_targets(wl, 10, seed=12)
    u = S.eval_field(x, xt)
    ref = -S.point_source_field(src, amp, xt)
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def _mutated_B(monkeypatch, S, kernel=None, weights=None, own_body=False):
    """Route B through the numpy sum with one slip planted."""
    import types
    orig_kernel = type(S).kernel

    def apply_B(self, sigma, rows=None):
        sig = np.asarray(sigma, dtype=np.complex128)
        vec = sig.ndim == 1
        sig = sig[:, None] if vec else sig
        w = self.w if weights is None else weights(self)
        with np.errstate(divide="ignore", invalid="ignore"):
            G = (kernel or orig_kernel)(self, self.x, self.x, self.n)
        G[~np.isfinite(G)] = 0.0
        if not own_body:
            G[self.body_of[:, None] == self.body_of[None, :]] = 0.0
        out = G @ (w[:, None] * sig)
        return out[:, 0] if vec else out
    monkeypatch.setattr(S, "apply_B", types.MethodType(apply_B, S))


def test_greens_identity_passes_with_the_numpy_sum(small_system, monkeypatch):
    wl, S = small_system
    _mutated_B(monkeypatch, S)
    e = _greens_error(S, wl)
    print(f"unmutated B: {e:.2e}")
    assert e < 1e-6


def test_inward_source_normals_in_B_fail(small_system, monkeypatch):
    wl, S = small_system
    orig = type(S).kernel
    _mutated_B(monkeypatch, S, kernel=lambda self, xt, xs, ns: orig(self, xt, xs, -ns))
    assert _greens_error(S, wl) > 1e-4


def test_B_without_weights_fails(small_system, monkeypatch):
    wl, S = small_system
    _mutated_B(monkeypatch, S, weights=lambda self: np.ones_like(self.w))
    assert _greens_error(S, wl) > 1e-4


def test_B_with_the_own_body_fails(small_system, monkeypatch):
    wl, S = small_system
    _mutated_B(monkeypatch, S, own_body=True)
    assert _greens_error(S, wl) > 1e-4
