"""Tile autotuner: choose the walk (`tile` of the lattice descriptor) per
lattice shape and precision by timing the library's own update kernels.

Candidates are plain checkerboard order (-1) and every z-strip width W that
divides Nz.  Each candidate runs one heat-bath sweep plus one overrelaxation
sweep on a scratch lattice (hot start, never the caller's lattice) after a
warm-up, timed with HIP events on the current stream; the fastest total
wins.  The walk changes no result, only the order in which blocks visit the
lattice, so tuning is safe to apply to any chain.  Choices are cached in a
JSON file keyed by device name, extents and precision.
"""
import json
import os

import torch

from . import (Lattice, su2_heatbath_sweep, su2_init_hot, su2_overrelax)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "su2_mi355x", "tiles.json")


def candidates(n):
    nz = int(n[2])
    return [-1] + [w for w in range(1, nz + 1) if nz % w == 0]


def _key(n, prec, device):
    name = torch.cuda.get_device_name(torch.device(device))
    return f"{name}|{'x'.join(str(int(v)) for v in n)}|{prec}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def measure(n, prec, tile, beta=2.3, reps=3, device="cuda"):
    """Milliseconds of (1 heat-bath + 1 overrelaxation sweep) with this walk."""
    lat = Lattice(n, prec, device=device, tile=tile)
    su2_init_hot(lat, 1)
    su2_heatbath_sweep(lat, beta, 1, 0)
    su2_overrelax(lat, 1)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for r in range(reps):
        torch.cuda.synchronize()
        t0.record()
        su2_heatbath_sweep(lat, beta, 1, 1 + r)
        su2_overrelax(lat, 1)
        t1.record()
        torch.cuda.synchronize()
        best = min(best, t0.elapsed_time(t1))
    return best


def tune(n, prec="f32", device="cuda", cache=DEFAULT_CACHE, reps=3, refresh=False, max_candidates=None):
    """Return the fastest tile for extents n (and store it in the cache)."""
    key = _key(n, prec, device)
    table = _load(cache) if cache else {}
    if not refresh and key in table:
        return int(table[key]["tile"])
    cands = candidates(n)
    if max_candidates is not None:
        cands = cands[:max_candidates]
    times = {t: measure(n, prec, t, reps=reps, device=device) for t in cands}
    best = min(times, key=times.get)
    if cache:
        table = _load(cache)
        table[key] = {"tile": best, "ms": times}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best
