"""Launch-shape autotuner for the stepping kernels.

For a grid class (padded rows, padded columns, shot count) every candidate
rows-per-wave value is timed with the library's event timer on a short
record (same grid and shots, few time steps), separately for the forward,
recompute, adjoint and Born steps, with one and with two time steps per
launch.  The fastest height per kernel is kept for each mode, and the mode
with the smaller time per gradient step (two forwards, as in an Anderson
iteration with one line-search trial, plus recompute and adjoint) wins.
The choice is cached in a JSON file.  Results are bitwise independent of it.
"""
from __future__ import annotations

import json
import os
import types

import numpy as np

CANDIDATES = (8, 12, 16, 20, 24, 28, 32, 40, 48, 64)
KERNELS = (0, 1, 2, 3)  # forward, recompute, adjoint, Born


def _short(geom, nt):
    g = types.SimpleNamespace(**{k: getattr(geom, k) for k in (
        "nz", "nx", "nb", "h", "dt", "vref", "refl", "vmax_bound", "src_iz", "src_ix", "rec_iz", "rec_ix")})
    g.nt = nt
    g.wavelet = np.asarray(geom.wavelet, np.float32)[:nt].copy()
    return g


def grid_key(geom) -> str:
    S = int(np.asarray(geom.src_iz).size)
    return f"{geom.nz + 2 * geom.nb}x{geom.nx + 2 * geom.nb}x{S}/tb"


def cache_path() -> str:
    base = os.environ.get("AAFWI_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "aafwi")
    return os.path.join(base, "tiles.json")


def tune(geom, m, candidates=CANDIDATES, nt=48, use_cache=True, verbose=False) -> dict:
    """Return {"tb": two steps per launch, kernel_id: rows_per_wave} for this
    grid class (m: device model)."""
    import torch

    from ._lib import Context
    key = grid_key(geom)
    path = cache_path()
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cached = json.load(f)
        if key in cached:
            return {(k if k == "tb" else int(k)): v for k, v in cached[key].items()}
    g = _short(geom, nt)
    best = {(tb, k): (float("inf"), 0) for tb in (False, True) for k in KERNELS}
    table = {}
    with Context(g, ckpt_every=nt) as ctx:
        r = torch.zeros(ctx.data_shape, device=m.device)
        dm = torch.zeros_like(m)
        for tb in (False, True):
            ctx.set_time_blocking(tb)
            for rows in candidates:
                if rows > g.nz + 2 * g.nb:
                    continue
                ctx.set_tile(rows)
                ctx.forward_model(m, keep_ckpt=True)  # warm
                ctx.kernel_timing(1)
                ctx.forward_model(m, keep_ckpt=True)
                ctx.adjoint_from_residual(r)
                if not tb:
                    ctx.born(m, dm)
                for k in KERNELS:
                    ms, cnt = ctx.kernel_timing_read(k)
                    if not cnt:
                        continue
                    per_step = ms / (2 if tb and k < 3 else 1)
                    table[(tb, rows, k)] = per_step
                    if per_step < best[(tb, k)][0]:
                        best[(tb, k)] = (per_step, rows)
                ctx.kernel_timing(0)
    cost = {tb: 2 * best[(tb, 0)][0] + best[(tb, 1)][0] + best[(tb, 2)][0] for tb in (False, True)}
    tb = cost[True] < cost[False]
    if verbose:
        for mode in (False, True):
            for k in KERNELS:
                row = " ".join(f"{rows}:{table[(mode, rows, k)] * 1e3:.1f}us" for rows in candidates
                               if (mode, rows, k) in table)
                if row:
                    print(f"autotune {key} {'two' if mode else 'one'}-step kernel {k} (per step): {row} "
                          f"-> {best[(mode, k)][1]}", flush=True)
        print(f"autotune {key}: per-step cost one-step {cost[False] * 1e3:.1f}us, two-step "
              f"{cost[True] * 1e3:.1f}us -> {'two' if tb else 'one'}-step", flush=True)
    out = {"tb": bool(tb)}
    for k in KERNELS:
        out[k] = best[(tb if k < 3 else False, k)][1]
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cached = {}
        if os.path.exists(path):
            with open(path) as f:
                cached = json.load(f)
        cached[key] = out
        with open(path, "w") as f:
            json.dump(cached, f, indent=1)
    return out


def apply(ctx, tiles: dict):
    if "tb" in tiles:
        ctx.set_time_blocking(bool(tiles["tb"]))
    for k, rows in tiles.items():
        if k != "tb":
            ctx.set_tile(int(rows), int(k))
