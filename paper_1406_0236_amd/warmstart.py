"""Learned warm start for the GMRES solve.

A small MLP maps (incident direction d, scaled wavenumber) to the low
azimuthal modes (|m| <= m_max) of the density on every contour node of every
body, with the incident phase at each body centre removed (so the targets
vary slowly with d and k).  It is trained on solves of the method itself,
produced by the library; training and inference run in the library's own
kernels (axs_mlp_*), and the prediction is decoded into an initial guess by
axs_density_from_modes.  axs_solve keeps the guess only if its FP64 residual
is below ||b||, so a poor prediction costs one operator application and no
accuracy.

The geometry is fixed and discretised once at the largest wavenumber of the
training range, so every sample has the same output size.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _lib
from ._lib import SOLVE_FP64, SOLVE_MIXED, Context, Mlp

K_MIN, K_MAX = 1.5 * math.pi, 2.5 * math.pi


def features(dirs, k, k_min=K_MIN, k_max=K_MAX):
    """Network input: the direction and the wavenumber mapped to [-1, 1]."""
    d = np.atleast_2d(dirs).astype(np.float64)
    kk = np.broadcast_to(np.asarray(k, dtype=np.float64), (d.shape[0],))
    ks = (2.0 * kk - (k_min + k_max)) / (k_max - k_min)
    return np.concatenate([d, ks[:, None]], axis=1).astype(np.float32)


def random_directions(n, rng):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def build_context(workload_at, k, autotune_cache=None):
    """Context (precomputed) of the workload at wavenumber k."""
    wl = workload_at(k)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return ctx, wl


def generate(workload_at, ks, dirs_per_k, mmax=8, tol=1e-8, log=None):
    """Solve every (k, direction) pair with the library and encode the solutions.

    Returns X (float32 [S, 4]) and Y (float32 [S, P]) as numpy arrays."""
    import torch
    Xs, Ys = [], []
    for i, (k, dirs) in enumerate(zip(ks, dirs_per_k)):
        t0 = time.time()
        ctx, _ = build_context(workload_at, k)
        v = ctx.incident_plane_waves(dirs)
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=tol, max_iters=100)
        coeff = _lib.modes_from_density(ctx, sol, dirs, mmax)
        Ys.append(coeff.cpu().numpy())
        Xs.append(features(dirs, k))
        ctx.close()
        del ctx, v, sol, coeff
        torch.cuda.empty_cache()
        if log:
            log(f"sample set {i + 1}/{len(ks)}: k = {k:.4f}, {len(dirs)} solves, "
                f"outer {max(x['iterations'] for x in info)}, {time.time() - t0:.2f} s")
    return np.concatenate(Xs), np.concatenate(Ys)


class WarmStart:
    """A trained warm-start network for one fixed geometry."""

    def __init__(self, ctx_for_device: Context, n_out: int, mmax=8, width=512, depth=4, seed=4):
        self.mmax = mmax
        self.width, self.depth = width, depth
        self.mlp = Mlp(ctx_for_device, 4, width, depth, n_out)
        rng = np.random.default_rng(seed)
        sizes = self.mlp.sizes
        flat = []
        for a, b in zip(sizes[:-1], sizes[1:]):
            flat.append(rng.standard_normal(a * b) * math.sqrt(2.0 / a))   # He initialisation
            flat.append(np.zeros(b))
        self.mlp.set_params(np.concatenate(flat))
        self.history = []

    def train(self, X, Y, epochs=200, batch=256, lr=1e-3, lr_final=1e-5, seed=5, log=None):
        """Adam on the mean squared error of the scaled targets; the scale is
        folded into the last layer at the end, so the raw network output is the
        mode vector."""
        import torch
        dev = f"cuda:{self.mlp.ctx.device}"
        scale = float(np.sqrt(np.mean(Y.astype(np.float64) ** 2))) or 1.0
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
        Yd = torch.from_numpy(np.ascontiguousarray(Y / scale, dtype=np.float32)).to(dev)
        S = Xd.shape[0]
        batch = min(batch, S)
        rng = np.random.default_rng(seed)
        steps_per_epoch = max(1, S // batch)
        total = epochs * steps_per_epoch
        t0 = time.time()
        step = 0
        for ep in range(epochs):
            perm = rng.permutation(S)[:steps_per_epoch * batch]
            # cosine decay from lr to lr_final over all steps
            t = np.arange(step, step + steps_per_epoch, dtype=np.float64)
            lrs = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * t / max(1, total - 1)))
            loss = self.mlp.train_epoch(Xd, Yd, perm, batch, lrs)
            step += steps_per_epoch
            self.history.append(loss)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log(f"epoch {ep + 1}/{epochs}: loss {loss:.4e} (scaled targets), {time.time() - t0:.1f} s")
        p = self.mlp.get_params().astype(np.float64)
        sizes = self.mlp.sizes
        off = sum(a * b + b for a, b in zip(sizes[:-2], sizes[1:-1]))
        p[off:] *= scale
        self.mlp.set_params(p)
        self.train_seconds = time.time() - t0
        return self.history

    def predict(self, ctx: Context, dirs, k):
        """Initial guess sigma0 (complex128 [nrhs][N]) for the context at wavenumber k."""
        import torch
        X = torch.from_numpy(features(dirs, k)).to(f"cuda:{ctx.device}")
        Y = self.mlp.forward(X)
        return _lib.density_from_modes(ctx, Y, dirs, self.mmax)


def evaluate(ws: WarmStart, workload_at, ks, dirs_per_k, tol=1e-7, log=None):
    """Held-out comparison: GMRES from the prediction vs from zero, per (k, direction)."""
    import torch
    rows = []
    for k, dirs in zip(ks, dirs_per_k):
        ctx, _ = build_context(workload_at, k)
        v = ctx.incident_plane_waves(dirs)
        sigma0 = ws.predict(ctx, dirs, k)
        out = {"k": float(k), "nrhs": len(dirs)}
        for mode, name in ((SOLVE_FP64, "fp64"), (SOLVE_MIXED, "mixed")):
            torch.cuda.synchronize()
            t0 = time.time()
            _, i0 = ctx.solve(v, mode=mode, tol=tol)
            torch.cuda.synchronize()
            t1 = time.time()
            _, i1 = ctx.solve(v, sigma0=sigma0, mode=mode, tol=tol)
            torch.cuda.synchronize()
            t2 = time.time()
            out[name] = {
                "zero_iters": float(np.mean([x["iterations"] for x in i0])),
                "warm_iters": float(np.mean([x["iterations"] for x in i1])),
                "zero_inner": float(np.mean([x["inner_iterations"] for x in i0])),
                "warm_inner": float(np.mean([x["inner_iterations"] for x in i1])),
                "zero_s": t1 - t0, "warm_s": t2 - t1,
                "warm_used": int(sum(x["used_warm_start"] for x in i1)),
                "converged": bool(all(x["converged"] for x in i0 + i1)),
            }
        # how good is the guess itself: the FP64 residual of sigma0 in the
        # preconditioned system, b - (sigma0 + D^{-1} B sigma0) with b = -D^{-1} v,
        # relative to ||b|| (1 for the zero guess); library applications,
        # norms on the host
        b = -ctx.apply_precond(v).cpu().numpy()
        r = b - ctx.apply_matvec(sigma0).cpu().numpy()
        rel = np.linalg.norm(r, axis=1) / np.linalg.norm(b, axis=1)
        out["guess_rel_residual"] = {"mean": float(np.mean(rel)), "min": float(np.min(rel)),
                                     "max": float(np.max(rel))}
        rows.append(out)
        if log:
            log(f"held-out k = {k:.4f}: guess residual {out['guess_rel_residual']['mean']:.3f} (mean), "
                f"fp64 iters {out['fp64']['zero_iters']:.1f} -> {out['fp64']['warm_iters']:.1f}, "
                f"mixed {out['mixed']['zero_s']:.3f} s -> {out['mixed']['warm_s']:.3f} s "
                f"(inner {out['mixed']['zero_inner']:.0f} -> {out['mixed']['warm_inner']:.0f})")
        ctx.close()
    return rows
