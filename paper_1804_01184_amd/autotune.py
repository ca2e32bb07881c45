"""Decomposition autotuner for the batched kernels.

The one-step adjoint kernel, the two-step adjoint kernel and the two-step
forward kernel have decompositions of their own (band rows swept per wave,
shots advanced together per wave, grid columns per lane), so they are tuned
separately on a short run of the real grid and shot count, with the whole
pressure history kept: each candidate is timed by its own launches, using
the library's per-launch HIP event timing.  The two-step adjoint shares the
shot groups (and so their partial gradients) with the one-step adjoint,
which then runs only for a leftover odd step of a segment; it is chosen
when its time per step beats the one-step kernel's.  The one-step forward
kernel (a leftover odd forward step) shares the one-step adjoint
decomposition.  Results are cached in a JSON file keyed by the shape and the
GPU; the package ships the results measured on MI355X for the benchmark
shapes (tuned_gfx950.json), consulted when the cache has none.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from .api import Grid, Plan

# band heights: every height from 8 to 16 (the kernels are bounded per CU,
# so how evenly the workgroups of a height spread over the CUs matters as
# much as the height), then coarser steps.  Each is lowered to the smallest
# height with the same number of bands (see balanced_rows).
ROWS = (8, 9, 10, 11, 12, 13, 14, 15, 16, 20, 24, 32, 48, 64, 96, 128)
ROWS2 = (12, 14, 16, 18, 20, 24, 28, 32, 48, 64, 96)
ROWSA = (12, 16, 20, 24, 32, 48, 64, 96, 128, 160, 192, 256)
# supported (shots per group, columns per lane) pairs of the one-step
# kernels and of the two-step forward kernel
PAIRS = ((1, 1), (2, 1), (4, 1), (8, 1), (1, 2), (2, 2), (4, 2), (1, 4), (2, 4))
PAIRS2 = ((1, 1), (2, 1), (1, 2), (2, 2), (1, 4))
PAIRSA = ((1, 1), (2, 1), (4, 1), (1, 2), (2, 2))


def strip_cols(cols, steps=1):
    """Output columns of one wave strip: 64 lanes less ceil(3 steps / cols)
    halo lanes on each side, times the columns per lane."""
    halo = (3 * steps + cols - 1) // cols
    return (64 - 2 * halo) * cols


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def cache_path():
    return os.environ.get("FWI2D_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fwi2d", "tune.json"))


def _key(Nz, Nx, S, npml, arch):
    return f"{arch}:{Nz}x{Nx}:S{S}:pml{npml}:v6"


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _waves(Nz, Nx, S, H, spg, cols, steps):
    strips = -(-Nx // strip_cols(cols, steps))
    return strips * -(-Nz // H) * -(-S // spg)


def balanced_rows(Nz, H):
    """The smallest band height giving as many bands of Nz rows as H does.
    A launch of a few rounds of waves lasts about as long as its tallest
    band, so with the band count fixed the last band should not be the
    short one: over 1081 rows, 192-row bands leave a last band of 121 rows
    and take as long as 181-row bands would with all six nearly equal."""
    bands = -(-Nz // H)
    return -(-Nz // bands)


def _triples(Nz, Nx, S, pairs, rows, steps):
    out = []
    rows = sorted({balanced_rows(Nz, H) for H in rows})
    for spg, cols in pairs:
        if spg > 1 and spg > 2 * S:
            continue
        mine = [(H, spg, cols) for H in rows
                if 512 <= _waves(Nz, Nx, S, H, spg, cols, steps) <= 65536]
        out += mine or [(min(rows), spg, cols)]
    return sorted(set(out))


def candidates(Nz, Nx, S):
    """(band_rows, shots_per_group, lane_cols) triples of the one-step
    kernels giving between 512 and 65536 waves."""
    return _triples(Nz, Nx, S, PAIRS, ROWS, 1)


def candidates2(Nz, Nx, S):
    """The same for the two-step forward kernel (halo of 6 rows and
    columns)."""
    return _triples(Nz, Nx, S, PAIRS2, ROWS2, 2)


def candidates_adj2(Nz, Nx, S):
    """The same for the two-step adjoint kernel."""
    return _triples(Nz, Nx, S, PAIRSA, ROWSA, 2)


def load_cache():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(c):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(c, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _probe_grid(grid, nt_probe):
    return Grid(grid.nz, grid.nx, grid.dz, grid.dx, grid.npml, nt_probe, grid.dt, grid.vmax,
                grid.pml_r)


def measure(grid: Grid, src_xz, rec_xz, nt_probe=24, reps=2, device=None, **decomp):
    """Device time (ms) per launch of each kernel class of a gradient over
    nt_probe steps with the decomposition `decomp` (Plan keywords)."""
    g = _probe_grid(grid, nt_probe)
    plan = Plan(g, src_xz, rec_xz, ckpt_every=nt_probe, device=device, **decomp)
    dev = plan.device
    K = torch.full((grid.nz, grid.nx), 2000.0 * 2000.0 ** 2, device=dev)
    rho = torch.full((grid.nz, grid.nx), 2000.0, device=dev)
    f = torch.zeros(nt_probe, device=dev)
    f[1] = 1.0
    adj = torch.ones((plan.nshots, plan.nrec, nt_probe), device=dev)
    plan.adjoint("k-rho", K, rho, f, adj)          # warm
    torch.cuda.synchronize(dev)
    plan.timing(True)
    for _ in range(reps):
        plan.adjoint("k-rho", K, rho, f, adj)
    t = plan.timing_read(reset=True)
    plan.timing(False)
    return {k: ms / n for k, (n, ms) in t.items() if n > 0}


def tune(grid: Grid, src_xz, rec_xz, force=False, verbose=False, device=None):
    """Plan keywords of the tuned decomposition for this shape (from the
    cache or by measuring): band_rows, shots_per_group, lane_cols of the
    one-step kernels and the two_step_* fields of the two-step kernel."""
    src = np.asarray(src_xz).reshape(-1, 2)
    S = src.shape[0]
    Nz, Nx = grid.padded
    key = _key(Nz, Nx, S, grid.npml, _arch())
    cache = load_cache()
    if not force and key in cache:
        return dict(cache[key]["best"])
    if not force:
        try:
            with open(SHIPPED) as fh:
                shipped = json.load(fh)
        except (OSError, ValueError):
            shipped = {}
        if key in shipped:
            return dict(shipped[key]["best"])
    t0 = time.perf_counter()
    res1, resa, res2 = [], [], []
    for H, spg, cols in candidates_adj2(Nz, Nx, S):
        t = measure(grid, src_xz, rec_xz, device=device, shots_per_group=spg, two_step=1,
                    adj_two_step=2, adj_two_step_band_rows=H, adj_two_step_lane_cols=cols)
        resa.append({"adj_two_step_band_rows": H, "shots_per_group": spg,
                     "adj_two_step_lane_cols": cols, "pair_ms": t.get("adj_pair", 0.0)})
        if verbose:
            print(f"  two-step adjoint band_rows={H:4d} spg={spg} cols={cols}: "
                  f"{resa[-1]['pair_ms'] * 1e3:8.1f} us per 2 steps", flush=True)
    # one-step adjoint: the shot grouping of the best pair (whose leftover
    # steps it takes) and the widest grouping (if the pair loses)
    spg_pair = min(resa, key=lambda r: r["pair_ms"])["shots_per_group"] if resa else 0
    for H, spg, cols in candidates(Nz, Nx, S):
        if spg not in (spg_pair, 8) and resa:
            continue
        t = measure(grid, src_xz, rec_xz, device=device, band_rows=H, shots_per_group=spg,
                    lane_cols=cols, two_step=1, adj_two_step=1)
        res1.append({"band_rows": H, "shots_per_group": spg, "lane_cols": cols,
                     "adj_ms": t.get("adj_step", 0.0), "fwd_ms": t.get("fwd_step", 0.0)})
        if verbose:
            print(f"  adjoint band_rows={H:4d} spg={spg} cols={cols}: "
                  f"{res1[-1]['adj_ms'] * 1e3:8.1f} us", flush=True)
    best1 = min(res1, key=lambda r: r["adj_ms"])
    best = {k: best1[k] for k in ("band_rows", "shots_per_group", "lane_cols")}
    best["adj_two_step"] = 1
    if resa:
        besta = min(resa, key=lambda r: r["pair_ms"])
        if besta["pair_ms"] < 2.0 * best1["adj_ms"]:
            # the one-step kernels take the pair's shot groups
            same = [r for r in res1 if r["shots_per_group"] == besta["shots_per_group"]]
            one = min(same, key=lambda r: r["adj_ms"]) if same else None
            best = {"band_rows": one["band_rows"] if one else 0,
                    "shots_per_group": besta["shots_per_group"],
                    "lane_cols": one["lane_cols"] if one else 1,
                    "adj_two_step": 2,
                    "adj_two_step_band_rows": besta["adj_two_step_band_rows"],
                    "adj_two_step_lane_cols": besta["adj_two_step_lane_cols"]}
    # with the two-step kernels the one-step kernels run only for a leftover
    # odd step: the two-step times decide
    for H, spg, cols in candidates2(Nz, Nx, S):
        t = measure(grid, src_xz, rec_xz, device=device, **best,
                    two_step=2, two_step_band_rows=H, two_step_shots_per_group=spg,
                    two_step_lane_cols=cols)
        if "fwd_pair" not in t:
            continue   # not available with this shot padding
        res2.append({"two_step_band_rows": H, "two_step_shots_per_group": spg,
                     "two_step_lane_cols": cols, "pair_ms": t["fwd_pair"]})
        if verbose:
            print(f"  two-step band_rows={H:4d} spg={spg} cols={cols}: "
                  f"{t['fwd_pair'] * 1e3:8.1f} us per 2 steps", flush=True)
    one_fwd = [r["fwd_ms"] for r in res1 if r["band_rows"] == best["band_rows"] and
               r["shots_per_group"] == best["shots_per_group"] and
               r["lane_cols"] == best["lane_cols"]]
    if res2:
        best2 = min(res2, key=lambda r: r["pair_ms"])
        if not one_fwd or best2["pair_ms"] < 2.0 * one_fwd[0]:
            best.update({k: best2[k] for k in ("two_step_band_rows", "two_step_shots_per_group",
                                               "two_step_lane_cols")})
            best["two_step"] = 2
        else:
            best["two_step"] = 1
    else:
        best["two_step"] = 1
    cache = load_cache()
    cache[key] = {"best": best, "adjoint": res1, "adj_two_step": resa, "two_step": res2,
                  "seconds": time.perf_counter() - t0}
    save_cache(cache)
    return dict(best)


def tuned_plan(grid: Grid, src_xz, rec_xz, **kw):
    """A batched Plan with the tuned decomposition."""
    best = tune(grid, src_xz, rec_xz, device=kw.get("device"))
    return Plan(grid, src_xz, rec_xz, **{**best, **kw})


__all__ = ["tune", "tuned_plan", "candidates", "candidates2", "candidates_adj2", "measure",
           "balanced_rows"]
