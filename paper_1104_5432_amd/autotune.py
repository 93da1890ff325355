"""Walk autotuner: choose the walk (`tile`, `tile_y` of the lattice
descriptor) per lattice shape and precision by timing the library's own
update kernels.

Candidates are plain checkerboard order (tile -1), every z-strip width W
that divides Nz, each with the columns split into S = 1, 2, 4 or 8 row
ranges (S dividing Ny), and the LDS-staged overrelaxation (tile -2) with
the other kernels' default strips in S row ranges.  Each candidate runs one
heat-bath sweep plus one overrelaxation sweep on a scratch lattice (hot
start, never the caller's lattice) after a warm-up, timed with HIP events on the current stream; the fastest total
wins.  The walk changes no result, only the order in which blocks visit the
lattice, so tuning is safe to apply to any chain.  Choices are cached in a
JSON file keyed by device architecture, CU count, extents and precision; a
table shipped with the package (tuned_walks.json, measured on an MI355X)
answers for the benchmarked lattices before anything is timed.
"""
import json
import os

import torch

from . import (Lattice, su2_heatbath_sweep, su2_init_hot, su2_overrelax)

# The cache file: $SU2_AUTOTUNE_CACHE, else ~/.cache/su2_mi355x/tiles.json.
DEFAULT_CACHE = os.environ.get("SU2_AUTOTUNE_CACHE") or os.path.join(
    os.path.expanduser("~"), ".cache", "su2_mi355x", "tiles.json")
# Walks measured on an MI355X for the benchmarked lattices (same key format);
# consulted after the cache and before any timing.
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_walks.json")


def candidates(n):
    """(tile, tile_y) pairs: plain order, then strip widths x row splits,
    then the LDS-staged overrelaxation (tile -2) with the heat bath's
    default strips split into row ranges."""
    ny, nz = int(n[1]), int(n[2])
    out = [(-1, 0)]
    for w in range(1, nz + 1):
        if nz % w:
            continue
        for sy in (1, 2, 4, 8):
            if ny % sy == 0:
                out.append((w, sy))
    for sy in (1, 2, 4, 8):
        if ny % sy == 0:
            out.append((-2, sy))
    return out


def _key(n, prec, device):
    # architecture and CU count: the marketing name can differ between
    # processes on the same device (e.g. under a profiler)
    p = torch.cuda.get_device_properties(torch.device(device))
    arch = (getattr(p, "gcnArchName", "") or p.name).split(":")[0]
    return key_for(arch, p.multi_processor_count, n, prec)


def key_for(arch, cus, n, prec):
    return f"{arch}|{int(cus)}cu|{'x'.join(str(int(v)) for v in n)}|{prec}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def measure(n, prec, walk, beta=2.3, reps=3, device="cuda"):
    """Milliseconds of (1 heat-bath + 1 overrelaxation sweep) with this walk."""
    tile, tile_y = walk
    lat = Lattice(n, prec, device=device, tile=tile, tile_y=tile_y)
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
    """Return the fastest walk (tile, tile_y) for extents n (and store it in
    the cache)."""
    key = _key(n, prec, device)
    if not refresh:
        for table in (_load(cache) if cache else {}, _load(SHIPPED)):
            if key in table and "tile_y" in table[key]:
                return int(table[key]["tile"]), int(table[key]["tile_y"])
    cands = candidates(n)
    if max_candidates is not None:
        cands = cands[:max_candidates]
    times = {c: measure(n, prec, c, reps=reps, device=device) for c in cands}
    best = min(times, key=times.get)
    if cache:
        table = _load(cache)
        table[key] = {"tile": best[0], "tile_y": best[1],
                      "ms": {f"{c[0]},{c[1]}": v for c, v in times.items()}}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best
