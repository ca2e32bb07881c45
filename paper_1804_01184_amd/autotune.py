"""Tile-shape / shot-group autotuner for the batched kernels.

For a problem shape (padded grid, shots) it times the batched forward and
adjoint step kernels of each candidate (tile rows, shot groups) on a short run
of the real grid and shot count, using the library's per-launch HIP event
timing, and keeps the configuration with the lowest cost of one gradient
time step (two forward-type steps — forward and recompute — plus one adjoint
step).  Results are cached in a JSON file keyed by the shape and the GPU.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import _lib as L
from .api import Grid, Plan

TILES = (8, 16, 32)


def cache_path():
    return os.environ.get("FWI2D_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fwi2d", "tune.json"))


def _key(Nz, Nx, S, npml, arch):
    return f"{arch}:{Nz}x{Nx}:S{S}:pml{npml}"


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def candidates(Nz, Nx, S):
    out = []
    for tz in TILES:
        ntiles = ((Nx + 63) // 64) * ((Nz + tz - 1) // tz)
        g = 1
        while g <= S:
            blocks = ntiles * g
            if 128 <= blocks <= 32768 or (g == 1 and blocks > 32768) or \
                    (g == S and blocks < 128):
                out.append((tz, g))
            g *= 2
        if S not in [c[1] for c in out if c[0] == tz] and 128 <= ntiles * S <= 32768:
            out.append((tz, S))
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


def measure(grid: Grid, src_xz, rec_xz, tile_z, groups, nt_probe=24, reps=2, device=None):
    """Per-step device time (ms) of the batched forward and adjoint kernels."""
    g = Grid(grid.nz, grid.nx, grid.dz, grid.dx, grid.npml, nt_probe, grid.dt, grid.vmax,
             grid.pml_r)
    plan = Plan(g, src_xz, rec_xz, tile_z=tile_z, shot_groups=groups,
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
    """(tile_z, shot_groups) for this shape, from the cache or by measuring."""
    src = np.asarray(src_xz).reshape(-1, 2)
    S = src.shape[0]
    Nz, Nx = grid.padded
    key = _key(Nz, Nx, S, grid.npml, _arch())
    cache = load_cache()
    if not force and key in cache:
        return tuple(cache[key]["best"])
    results = []
    t0 = time.perf_counter()
    for tz, G in candidates(Nz, Nx, S):
        fwd, adj = measure(grid, src_xz, rec_xz, tz, G, device=device)
        cost = 2.0 * fwd + adj
        results.append({"tile_z": tz, "groups": G, "fwd_ms": fwd, "adj_ms": adj, "cost": cost})
        if verbose:
            print(f"  tile_z={tz:2d} groups={G:3d}: fwd {fwd * 1e3:8.1f} us  "
                  f"adj {adj * 1e3:8.1f} us", flush=True)
    best = min(results, key=lambda r: r["cost"])
    cache = load_cache()
    cache[key] = {"best": [best["tile_z"], best["groups"]], "results": results,
                  "seconds": time.perf_counter() - t0}
    save_cache(cache)
    return best["tile_z"], best["groups"]


def tuned_plan(grid: Grid, src_xz, rec_xz, **kw):
    """A batched Plan with the tuned tile shape and shot groups."""
    tz, G = tune(grid, src_xz, rec_xz, device=kw.get("device"))
    return Plan(grid, src_xz, rec_xz, tile_z=tz, shot_groups=G, **kw)


__all__ = ["tune", "tuned_plan", "candidates", "measure", "L"]
