"""Launch-shape autotuner for the stepping kernels.

For a grid class (padded rows, padded columns, shot count) every candidate
rows-per-wave value is timed with the library's event timer on a short
record (same grid and shots, few time steps), separately for the forward,
recompute, adjoint and Born steps, with one and with two time steps per
launch and with both tile orders (x-tiles of a strip adjacent, or strips of
a column adjacent).  Per kernel the fastest (mode, height, order) per time
step is kept, ties within 2 % going to the tallest strips; the forward, recompute and adjoint choose their modes
independently.  The choice is cached in a JSON file; shapes measured on
MI355X for the common grid classes ship with the package (a tuning table
like a library's performance database) and are used when the user cache has
no entry, so that runs on fresh machines take the same launch shape.
Results are bitwise independent of the shape.
"""
from __future__ import annotations

import json
import os
import types

import numpy as np

CANDIDATES = (8, 12, 16, 20, 24, 28, 32, 40, 48, 64)
CANDIDATES_TWO = (16, 20, 24, 32, 40, 48, 64, 80, 96, 120)  # two-step launches (strips up to 120 rows)
KERNELS = (0, 1, 2, 3)  # forward, recompute, adjoint, Born
TIE = 0.02


def _short(geom, nt):
    g = types.SimpleNamespace(**{k: getattr(geom, k) for k in (
        "nz", "nx", "nb", "h", "dt", "vref", "refl", "vmax_bound", "src_iz", "src_ix", "rec_iz", "rec_ix")})
    g.nt = nt
    g.wavelet = np.asarray(geom.wavelet, np.float32)[:nt].copy()
    return g


def grid_key(geom) -> str:
    S = int(np.asarray(geom.src_iz).size)
    return f"{geom.nz + 2 * geom.nb}x{geom.nx + 2 * geom.nb}x{S}/mode-order-120"


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def _lookup(path, key):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cached = json.load(f)
    if key not in cached:
        return None
    return {(k if not k.isdigit() else int(k)): v for k, v in cached[key].items()}


def cache_path() -> str:
    base = os.environ.get("AAFWI_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "aafwi")
    return os.path.join(base, "tiles.json")


def tune(geom, m, candidates=CANDIDATES, nt=48, use_cache=True, verbose=False) -> dict:
    """Return {kernel_id: rows per wave, "order<k>": tile order, "two<k>":
    two steps per launch (k < 3)} for this grid class (m: device model).
    With use_cache the user cache, then the shipped table, is consulted
    before timing anything; use_cache=False always times and stores nothing."""
    import torch

    from ._lib import Context
    key = grid_key(geom)
    path = cache_path()
    if use_cache:
        for p in (path, SHIPPED):
            hit = _lookup(p, key)
            if hit is not None:
                if verbose:
                    print(f"autotune {key}: launch shape from {p}", flush=True)
                return hit
    g = _short(geom, nt)
    best = {(tb, k): (float("inf"), 0, 0) for tb in (False, True) for k in KERNELS}
    table = {}
    with Context(g, ckpt_every=nt) as ctx:
        r = torch.zeros(ctx.data_shape, device=m.device)
        dm = torch.zeros_like(m)
        shapes = [(tb, order, rows) for tb in (False, True) for order in (0, 1)
                  for rows in (CANDIDATES_TWO if tb and candidates is CANDIDATES else candidates)
                  if rows <= g.nz + 2 * g.nb]
        for tb, order, rows in shapes:
            ctx.set_time_blocking(tb)
            ctx.set_tile_order(order)
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
                table[(tb, order, rows, k)] = per_step
                if per_step < best[(tb, k)][0]:
                    best[(tb, k)] = (per_step, rows, order)
            ctx.kernel_timing(0)
    if verbose:
        for mode in (False, True):
            for k in KERNELS:
                for order in (0, 1):
                    row = " ".join(f"{rows}:{table[(mode, order, rows, k)] * 1e3:.1f}us"
                                   for rows in sorted(set(candidates) | set(CANDIDATES_TWO))
                                   if (mode, order, rows, k) in table)
                    if row:
                        print(f"autotune {key} {'two' if mode else 'one'}-step kernel {k} order {order} (per step): "
                              f"{row}", flush=True)
    # within TIE of the fastest shape of a mode, take the tallest strips:
    # the same speed within timing noise, less halo re-reading
    for (tb, k), (t_best, _, _) in list(best.items()):
        near = [(rows, -order, order) for (tb2, order, rows, k2), per in table.items()
                if tb2 == tb and k2 == k and per <= t_best * (1 + TIE)]
        if near:
            rows, _, order = max(near)
            best[(tb, k)] = (table[(tb, order, rows, k)], rows, order)
    out = {}
    for k in KERNELS:
        two = k < 3 and best[(True, k)][0] < best[(False, k)][0]
        t, rows, order = best[(two, k)]
        out[k], out[f"order{k}"] = rows, order
        if k < 3:
            out[f"two{k}"] = bool(two)
            # the best height of each mode, for batches whose mode is fixed
            out[f"rows_one{k}"], out[f"rows_two{k}"] = best[(False, k)][1], best[(True, k)][1]
        if verbose:
            print(f"autotune {key} kernel {k}: {'two' if two else 'one'}-step, rows {rows}, order {order}, "
                  f"{t * 1e3:.1f} us per step", flush=True)
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
    """Set the launch modes, strip heights and tile orders of a tune() result."""
    for k in KERNELS:
        if f"two{k}" in tiles:
            ctx.set_time_blocking(bool(tiles[f"two{k}"]), k)
        if k in tiles:
            ctx.set_tile(int(tiles[k]), k)
        if f"order{k}" in tiles:
            ctx.set_tile_order(int(tiles[f"order{k}"]), k)


def class_rows(entry: dict, k: int, two: bool) -> int:
    """Strip height of kernel k for a launch mode from a tune() entry; 0 (the
    library default) when the entry holds no height for that mode."""
    if k < 3 and f"rows_{'two' if two else 'one'}{k}" in entry:
        return int(entry[f"rows_{'two' if two else 'one'}{k}"])
    if k == 3 or bool(entry.get(f"two{k}", False)) == two:
        return int(entry.get(k, 0))
    return 0


def tune_batch(batch, geoms, models, shots: int = 8, use_cache=True, verbose=False) -> dict:
    """Per-grid-class strip heights for a batch of uneven instances.

    Instances with the same padded grid form a class; each class is tuned
    once (tune() on its first instance with at most ``shots`` shots, from the
    caches when they hold it) and every instance of the class takes that
    class's height for the batch's own launch mode (one mode per kernel is
    shared by the whole batch, since one launch covers every instance).
    Returns {class key: {kernel: rows}}."""
    mask = batch.time_blocking()
    chosen = {}
    for i, (g, m) in enumerate(zip(geoms, models)):
        cls = (g.nz + 2 * g.nb, g.nx + 2 * g.nb)
        if cls not in chosen:
            S = int(np.asarray(g.src_iz).size)
            sub = g.subset_shots(list(range(min(S, shots)))) if hasattr(g, "subset_shots") else g
            entry = tune(sub, m, use_cache=use_cache, verbose=verbose)
            chosen[cls] = {k: class_rows(entry, k, bool(mask >> k & 1) if k < 3 else False) for k in KERNELS}
        for k, rows in chosen[cls].items():
            batch.set_instance_tile(i, rows, k)
    if verbose:
        print(f"autotune batch: per-class heights {chosen} (modes {mask})", flush=True)
    return {f"{a}x{b}": v for (a, b), v in chosen.items()}


def tune_in_place(ctx, m, d_obs=None, rows_one=(8, 16, 32, 64), rows_two=(16, 24, 48, 96), orders=(0, 1),
                  verbose=False) -> dict:
    """Launch shapes timed where the run happens: on the caller's own context
    (its grid, shots, record length and checkpoint layout), its model and,
    with ``d_obs``, its own residual, so that the planes the kernels stream
    hold the values of the real run (a short record from rest holds mostly
    zeros).  Every candidate (steps per launch, tile order, strip height) is
    applied to the forward, recompute and adjoint kernels at once and timed
    over one forward run with kept checkpoints and one backward pass of the
    whole record; per kernel the fastest per-step time wins (ties within 2 %
    to the taller strip).  The Born kernel keeps the context's setting.
    Returns a tune()-style entry for the three kernels (apply() takes it) and
    leaves the context in that shape."""
    import torch
    d = ctx._new(ctx.data_shape)
    r = ctx._new(ctx.data_shape)
    J = ctx._new((1,), torch.float64)
    table = {}
    shapes = [(False, o, h) for o in orders for h in rows_one] + [(True, o, h) for o in orders for h in rows_two]
    for tb, order, rows in shapes:
        if rows > ctx.nz + 2 * ctx.nb and rows != min(rows_one + rows_two):
            continue
        for k in range(3):
            ctx.set_time_blocking(tb, k)
            ctx.set_tile_order(order, k)
            ctx.set_tile(rows, k)
        ctx.kernel_timing(1)
        ctx.forward_model(m, d, keep_ckpt=True)
        if d_obs is not None:
            ctx.residual_misfit(d, d_obs, r, J)
        else:
            r.copy_(d)
        ctx.adjoint_from_residual(r)
        for k in range(3):
            ms, cnt = ctx.kernel_timing_read(k)
            if cnt:
                table[(tb, order, rows, k)] = ms / (2 if tb else 1)
        ctx.kernel_timing(0)
        if verbose:
            print(f"autotune in place: {'two' if tb else 'one'}-step order {order} rows {rows}: "
                  + ", ".join(f"k{k} {table.get((tb, order, rows, k), float('nan')) * 1e3:.1f} us/step"
                              for k in range(3)), flush=True)
    out = {}
    for k in range(3):
        cand = {key: t for key, t in table.items() if key[3] == k}
        best = min(cand.values())
        near = [(key[2], -key[1], key) for key, t in cand.items() if t <= best * (1 + TIE)]
        # the best mode first, then within that mode the tallest strip inside the tie band
        mode = min(cand, key=cand.get)[0]
        near = [x for x in near if x[2][0] == mode] or near
        tb, order, rows, _ = max(near)[2]
        out[k], out[f"order{k}"], out[f"two{k}"] = rows, order, bool(tb)
        for mm in (False, True):
            mc = {key: t for key, t in cand.items() if key[0] == mm}
            if mc:
                out[f"rows_{'two' if mm else 'one'}{k}"] = min(mc, key=mc.get)[2]
        if verbose:
            print(f"autotune in place: kernel {k}: {'two' if tb else 'one'}-step, rows {rows}, order {order}, "
                  f"{cand[(tb, order, rows, k)] * 1e3:.1f} us per step", flush=True)
    apply(ctx, out)
    return out
