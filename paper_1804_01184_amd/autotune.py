"""Decomposition autotuner for the batched kernels.

For a problem shape (padded grid, shots) it times the batched forward and
adjoint step kernels of each candidate (band rows swept per wave, shots
advanced together per wave, grid columns per lane) on a short run of the
real grid and shot count,
using the library's per-launch HIP event timing, and keeps the configuration
with the lowest cost of one gradient time step (two forward-type steps —
forward and recompute — plus one adjoint step).  Results are cached in a JSON
file keyed by the shape and the GPU.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import _lib as L
from .api import Grid, Plan

ROWS = (8, 12, 16, 24, 32, 48, 64, 96, 128)
# supported (shots per group, columns per lane) pairs
PAIRS = ((1, 1), (2, 1), (4, 1), (8, 1), (1, 2), (2, 2), (4, 2), (1, 4), (2, 4))


def strip_cols(cols):
    """Output columns of one wave strip: 64 lanes less ceil(3 / cols) halo
    lanes on each side, times the columns per lane."""
    halo = (3 + cols - 1) // cols
    return (64 - 2 * halo) * cols


def cache_path():
    return os.environ.get("FWI2D_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fwi2d", "tune.json"))


def _key(Nz, Nx, S, npml, arch):
    return f"{arch}:{Nz}x{Nx}:S{S}:pml{npml}:v2"


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def candidates(Nz, Nx, S):
    """(band_rows, shots_per_group, lane_cols) triples giving between 512
    and 65536 waves."""
    out = []
    for spg, cols in PAIRS:
        if spg > 1 and spg > 2 * S:
            continue
        strips = (Nx + strip_cols(cols) - 1) // strip_cols(cols)
        groups = (S + spg - 1) // spg
        mine = []
        for H in ROWS:
            waves = strips * ((Nz + H - 1) // H) * groups
            if 512 <= waves <= 65536:
                mine.append((H, spg, cols))
        out += mine or [(min(ROWS), spg, cols)]
    return sorted(set(out))


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


def measure(grid: Grid, src_xz, rec_xz, band_rows, spg, cols=1, nt_probe=24, reps=2,
            device=None):
    """Per-step device time (ms) of the batched forward and adjoint kernels."""
    g = Grid(grid.nz, grid.nx, grid.dz, grid.dx, grid.npml, nt_probe, grid.dt, grid.vmax,
             grid.pml_r)
    plan = Plan(g, src_xz, rec_xz, band_rows=band_rows, shots_per_group=spg, lane_cols=cols,
                ckpt_every=max(2, nt_probe // 4), device=device)
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
    fwd = t["fwd_step"][1] / max(1, t["fwd_step"][0])
    adj_ms = t["adj_step"][1] / max(1, t["adj_step"][0])
    return fwd, adj_ms


def tune(grid: Grid, src_xz, rec_xz, force=False, verbose=False, device=None):
    """(band_rows, shots_per_group, lane_cols) for this shape, from the cache
    or by measuring."""
    src = np.asarray(src_xz).reshape(-1, 2)
    S = src.shape[0]
    Nz, Nx = grid.padded
    key = _key(Nz, Nx, S, grid.npml, _arch())
    cache = load_cache()
    if not force and key in cache:
        return tuple(cache[key]["best"])
    results = []
    t0 = time.perf_counter()
    for H, spg, cols in candidates(Nz, Nx, S):
        fwd, adj = measure(grid, src_xz, rec_xz, H, spg, cols, device=device)
        cost = 2.0 * fwd + adj
        results.append({"band_rows": H, "spg": spg, "cols": cols, "fwd_ms": fwd,
                        "adj_ms": adj, "cost": cost})
        if verbose:
            print(f"  band_rows={H:4d} spg={spg} cols={cols}: fwd {fwd * 1e3:8.1f} us  "
                  f"adj {adj * 1e3:8.1f} us", flush=True)
    best = min(results, key=lambda r: r["cost"])
    cache = load_cache()
    cache[key] = {"best": [best["band_rows"], best["spg"], best["cols"]], "results": results,
                  "seconds": time.perf_counter() - t0}
    save_cache(cache)
    return best["band_rows"], best["spg"], best["cols"]


def tuned_plan(grid: Grid, src_xz, rec_xz, **kw):
    """A batched Plan with the tuned decomposition."""
    H, spg, cols = tune(grid, src_xz, rec_xz, device=kw.get("device"))
    return Plan(grid, src_xz, rec_xz, band_rows=H, shots_per_group=spg, lane_cols=cols, **kw)


__all__ = ["tune", "tuned_plan", "candidates", "measure", "L"]
