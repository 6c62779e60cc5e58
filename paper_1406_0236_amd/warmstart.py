"""Learned warm start for the GMRES solve: orchestration of library calls.

The library (include/axs.h, axs_mlp_* and axs_warm_start_*) does every step:
it encodes the method's own solutions into training targets (the
multiple-scattering part of the density, split by source body, phases taken
out), trains the network (feature and target scaling, permutation, cosine
learning rate, Adam, the scale folded into the last layer), and predicts an
initial guess sigma0 = b~ + decoded network output, b~ = -D^{-1} v.  This
module only loops over wavenumbers, moves tensors between calls and times
the solves it compares.

The geometry is fixed and discretised once at the largest wavenumber of the
training range, so every sample has the same output size.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _lib
from ._lib import FP64, SOLVE_FP64, SOLVE_MIXED, Context, Mlp

K_MIN, K_MAX = 1.5 * math.pi, 2.5 * math.pi


def random_directions(n, rng):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def build_context(workload_at, k):
    """Context (precomputed) of the workload at wavenumber k."""
    wl = workload_at(k)
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    return ctx, wl


def generate(workload_at, ks, dirs_per_k, mmax=8, tol=1e-8, log=None):
    """Solve every (k, direction) pair with the library and encode the solutions.

    Returns X (float32 [S, 4] = (d, k)) and Y (float32 [S, P]) as numpy arrays."""
    import torch
    Xs, Ys = [], []
    for i, (k, dirs) in enumerate(zip(ks, dirs_per_k)):
        t0 = time.time()
        ctx, _ = build_context(workload_at, k)
        v = ctx.incident_plane_waves(dirs)
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=tol, max_iters=100)
        Ys.append(_lib.warm_start_encode(ctx, sol, dirs, mmax).cpu().numpy())
        Xs.append(np.concatenate([dirs, np.full((len(dirs), 1), k)], axis=1).astype(np.float32))
        ctx.close()
        del ctx, v, sol
        torch.cuda.empty_cache()
        if log:
            log(f"sample set {i + 1}/{len(ks)}: k = {k:.4f}, {len(dirs)} solves, "
                f"outer {max(x['iterations'] for x in info)}, {time.time() - t0:.2f} s")
    return np.concatenate(Xs), np.concatenate(Ys)


class WarmStart:
    """A trained warm-start network for one fixed geometry."""

    def __init__(self, ctx_for_device: Context, n_out: int, width=512, depth=4, k_range=(K_MIN, K_MAX)):
        self.width, self.depth = width, depth
        self.k_range = (float(k_range[0]), float(k_range[1]))
        self.mlp = Mlp(ctx_for_device, 4, width, depth, n_out)
        self.history = []

    def train(self, X, Y, epochs=200, batch=256, lr=1e-3, lr_final=1e-5, seed=5, init_seed=4, log=None):
        """axs_mlp_train on the samples (numpy X [S, 4], Y [S, P])."""
        import torch
        dev = f"cuda:{self.mlp.ctx.device}"
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
        Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(dev)
        t0 = time.time()
        hp = {"epochs": epochs, "batch": batch, "lr": lr, "lr_final": lr_final, "seed": seed,
              "init_seed": init_seed, "k_min": self.k_range[0], "k_max": self.k_range[1]}
        self.history = [float(x) for x in _lib.mlp_train(self.mlp, Xd, Yd, hp)]
        self.train_seconds = time.time() - t0
        if log:
            log(f"trained {epochs} epochs in {self.train_seconds:.1f} s: loss {self.history[0]:.4e} -> "
                f"{self.history[-1]:.4e} (scaled targets)")
        return self.history

    def predict(self, ctx: Context, dirs):
        """axs_mlp_predict: initial guess (complex128 [nrhs][N]) on ctx for the plane waves dirs."""
        return _lib.mlp_predict(self.mlp, ctx, dirs, self.k_range)


def _residual(ctx, b, x):
    """||b - (x + D^{-1} B x)|| / ||b|| per rhs (library operator, norms for the report)."""
    import torch
    r = b - ctx.apply_matvec(x, FP64)
    return (torch.linalg.norm(r, dim=1) / torch.linalg.norm(b, dim=1)).cpu().numpy()


def evaluate(ws: WarmStart, workload_at, ks, dirs_per_k, tol=1e-7, log=None):
    """Held-out comparison of three initial guesses per (k, direction): zero,
    the single-body responses b~ = -D^{-1} v, and the learned guess b~ + network;
    FP64 GMRES and the mixed solver from each, iterations and seconds."""
    import torch
    rows = []
    for k, dirs in zip(ks, dirs_per_k):
        ctx, _ = build_context(workload_at, k)
        v = ctx.incident_plane_waves(dirs)
        b = -ctx.apply_precond(v, FP64)
        torch.cuda.synchronize()
        t0 = time.time()
        learned = ws.predict(ctx, dirs)
        torch.cuda.synchronize()
        t_pred = time.time() - t0
        guesses = {"zero": None, "single_body": b, "learned": learned}
        out = {"k": float(k), "nrhs": len(dirs), "predict_s": t_pred, "guess_rel_residual": {}}
        for name, g in guesses.items():
            rel = np.ones(len(dirs)) if g is None else _residual(ctx, b, g)
            out["guess_rel_residual"][name] = {"mean": float(np.mean(rel)), "max": float(np.max(rel))}
        for mode, mname in ((SOLVE_FP64, "fp64"), (SOLVE_MIXED, "mixed")):
            res = {}
            for name, g in guesses.items():
                ctx.solve(v, sigma0=g, mode=mode, tol=tol)        # warm-up of this path
                torch.cuda.synchronize()
                t0 = time.time()
                _, inf = ctx.solve(v, sigma0=g, mode=mode, tol=tol)
                torch.cuda.synchronize()
                dt = time.time() - t0
                res[name] = {"s": dt + (t_pred if name == "learned" else 0.0),
                             "iters": float(np.mean([x["iterations"] for x in inf])),
                             "inner": float(np.mean([x["inner_iterations"] for x in inf])),
                             "used": int(sum(x["used_warm_start"] for x in inf)),
                             "converged": bool(all(x["converged"] for x in inf))}
            out[mname] = res
        rows.append(out)
        if log:
            g = out["guess_rel_residual"]
            log(f"held-out k = {k:.4f}: guess residual zero 1, single-body {g['single_body']['mean']:.3f}, "
                f"learned {g['learned']['mean']:.3f}; fp64 iterations "
                + ", ".join(f"{n} {out['fp64'][n]['iters']:.1f}" for n in guesses)
                + "; mixed s " + ", ".join(f"{n} {out['mixed'][n]['s']:.3f}" for n in guesses))
        ctx.close()
    return rows


def summarise(rows):
    """Means over the held-out rows, per guess: residual of the guess, FP64 and
    mixed iterations and seconds (the learned guess's seconds include its prediction)."""
    out = {}
    for name in ("zero", "single_body", "learned"):
        out[name] = {
            "guess_rel_residual": float(np.mean([r["guess_rel_residual"][name]["mean"] for r in rows])),
            "fp64_iters": float(np.mean([r["fp64"][name]["iters"] for r in rows])),
            "fp64_s": float(np.mean([r["fp64"][name]["s"] for r in rows])),
            "mixed_outer": float(np.mean([r["mixed"][name]["iters"] for r in rows])),
            "mixed_inner": float(np.mean([r["mixed"][name]["inner"] for r in rows])),
            "mixed_s": float(np.mean([r["mixed"][name]["s"] for r in rows])),
            "converged": bool(all(r[m][name]["converged"] for r in rows for m in ("fp64", "mixed"))),
        }
    return out
