"""Launch-shape autotuner for the inter-body sum.

Sweeps the source order (points / rings), targets per thread, block size and
number of source splits on the live context, timing each candidate with the
library's HIP events on its own stream, and keeps the fastest.  Results are
cached in a JSON file keyed by (GPU architecture, precision, right-hand-side
count, unknowns bucket, largest N_F), so a later context with the same key
reuses the choice without re-timing.  Every candidate computes the same sum
(the parity tests check all supported shapes), so tuning never changes
results beyond rounding.
"""
from __future__ import annotations

import json
import math
import os

from ._lib import FP32, FP64, AxsError

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

CANDIDATES = [
    # (variant, targets per thread, block); the point and ring orders take the
    # right-hand sides in groups of up to 8, the MFMA orders in groups of 16 and
    # 1, 2 or 4 groups of 16 targets per wavefront (variant 4, the FP16
    # multiply-accumulate, is FP32 only and needs bodies whose bounding balls
    # do not overlap)
    (4, 2, 256), (4, 1, 256), (4, 4, 256),
    (3, 2, 256), (3, 1, 256), (3, 4, 256),
    (2, 4, 256), (2, 2, 256), (2, 8, 256), (2, 4, 128), (2, 2, 128), (2, 1, 128), (2, 1, 256),
    (1, 4, 256), (1, 2, 256), (1, 8, 256),
]
SPLITS = (0, 4, 16, 64)


def _arch(device):
    import torch
    try:
        return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(ctx, precision, nrhs, max_nf):
    bucket = 1 << max(0, int(math.ceil(math.log2(max(ctx.N, 1)))))
    return f"{_arch(ctx.device)}|{'fp32' if precision == FP32 else 'fp64'}|r{nrhs}|N{bucket}|nf{max_nf}"


def _time_candidate(ctx, x, precision, reps):
    best = float("inf")
    for _ in range(reps):
        ctx.apply_interbody(x, precision)
        best = min(best, ctx.last_timing()["interbody"])
    return best


def tune(ctx, precision, nrhs, max_nf, x=None, reps=2, cache_path=DEFAULT_CACHE, budget_ms=None,
         verbose=False):
    """Pick and apply the fastest inter-body launch shape for (precision, nrhs).

    ctx: a precomputed Context; max_nf: the largest N_F of its bodies (ring
    variant needs N_F <= block).  Returns (config, timings)."""
    import torch
    key = cache_key(ctx, precision, nrhs, max_nf)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        cfg = cache[key]["config"]
        ctx.set_interbody_config(precision, *cfg)
        return cfg, cache[key].get("timings_ms", {})
    if x is None:
        g = torch.Generator(device=f"cuda:{ctx.device}").manual_seed(1234)
        x = torch.randn((nrhs, ctx.N), dtype=torch.complex128, device=f"cuda:{ctx.device}", generator=g)
    ctx.set_timing(True)
    timings = {}
    spent = 0.0
    try:
        for variant, tpt, block in CANDIDATES:
            if variant == 2 and max_nf > block:
                continue
            if variant >= 3 and not (ctx.kappa or 0) > 0:
                continue
            if variant == 4 and (precision != FP32 or nrhs < 16):
                continue
            for splits in SPLITS:
                cfg = (variant, tpt, block, splits)
                ctx.set_interbody_config(precision, *cfg)
                try:
                    ms = _time_candidate(ctx, x, precision, reps)
                except AxsError:
                    # a shape this context cannot run (the library says why)
                    break
                timings[",".join(map(str, cfg))] = ms
                spent += ms * (reps + 1)
                if verbose:
                    print(f"[autotune] {key} {cfg}: {ms:.3f} ms", flush=True)
                if budget_ms is not None and spent > budget_ms:
                    break
            if budget_ms is not None and spent > budget_ms:
                break
    finally:
        ctx.set_timing(False)
    best = min(timings, key=timings.get)
    cfg = [int(v) for v in best.split(",")]
    ctx.set_interbody_config(precision, *cfg)
    if cache_path:
        cache[key] = {"config": cfg, "ms": timings[best], "timings_ms": timings}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return cfg, timings
