"""Learned block proposal: training on heat-bath configurations and chains
that interleave it with the heat bath.  Every step runs in the library's
kernels (su2_lp_* and the heat-bath/overrelaxation/observable entry points);
this module only sequences the calls.

- train(): a heat-bath chain generates configurations; after each sweep the
  network's maximum-likelihood gradient on that configuration is taken and
  one Adam step applied (the loss is the mean negative log density of every
  temporal link under its block proposal, which in equilibrium is minimised
  by the exact block marginal).
- run_chain(): n sweeps of 1 heat bath (+ n_or overrelaxation) and, when
  params are given, one learned sweep (network forward once, then the 16
  block classes); records the Polyakov loop, the plaquette, the acceptance
  and the wall time.
"""
import math
import time

import torch

from . import (Lattice, LPWork, su2_heatbath_sweep, su2_init_hot, su2_lp_adam, su2_lp_forward,
               su2_lp_loss_grad, su2_lp_param_count, su2_lp_sweep, su2_overrelax, su2_plaquette,
               su2_polyakov)

# parameter blocks: (name, number, fan_in) in the ABI's order
BLOCKS = [("W1", 27 * 8 * 32, 27 * 8), ("b1", 32, 0), ("W2", 27 * 32 * 32, 27 * 32), ("b2", 32, 0),
          ("W3", 27 * 32 * 32, 27 * 32), ("b3", 32, 0), ("V", 6 * 32, 0), ("bv", 6, 0)]


def init_params(seed, device="cuda"):
    """Convolution weights uniform in +-1/sqrt(fan_in); biases and the head
    zero, so an untrained network gives y = 0: the mean-field proposal."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    parts = []
    for _, count, fan in BLOCKS:
        if fan:
            parts.append((torch.rand(count, generator=g, dtype=torch.float64) * 2 - 1) / math.sqrt(fan))
        else:
            parts.append(torch.zeros(count, dtype=torch.float64))
    p = torch.cat(parts).to(torch.float32)
    assert p.numel() == su2_lp_param_count()
    return p.to(device)


def train(lat, beta, seed, n_configs, params=None, lr=2e-3, n_or=0, first_sweep=0, lpwork=None,
          log_every=0):
    """Train on n_configs successive heat-bath configurations of `lat` (which
    should be thermalised).  Returns (params, list of losses)."""
    dev = lat.device
    if params is None:
        params = init_params(seed, dev)
    lpwork = lpwork or LPWork(lat.n, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.empty(n_configs, dtype=torch.float64, device=dev)
    for k in range(n_configs):
        su2_heatbath_sweep(lat, beta, seed, first_sweep + k)
        if n_or:
            su2_overrelax(lat, n_or)
        su2_lp_loss_grad(lat, beta, params, lpwork, grad, loss[k:k + 1])
        su2_lp_adam(params, grad, m, v, k + 1, lr=lr)
        if log_every and (k + 1) % log_every == 0:
            torch.cuda.synchronize()
            print(f"train {k + 1}/{n_configs}: loss {loss[max(0, k - log_every + 1):k + 1].mean().item():.6f}",
                  flush=True)
    torch.cuda.synchronize()
    return params, loss.cpu().tolist()


def run_chain(lat, beta, seed, n_sweeps, params=None, n_or=0, first_sweep=0, lp_seed=None, lpwork=None):
    """Run and measure a chain; returns a dict of host lists and timings."""
    dev = lat.device
    poly = torch.empty((n_sweeps, 2), dtype=torch.float64, device=dev)
    plaq = torch.empty((n_sweeps, 7), dtype=torch.float64, device=dev)
    acc = torch.zeros(1, dtype=torch.int32, device=dev)
    y = torch.empty(lat.volume * 6, dtype=torch.float32, device=dev) if params is not None else None
    lpwork = (lpwork or LPWork(lat.n, dev)) if params is not None else None
    lp_seed = seed + 1 if lp_seed is None else lp_seed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_sweeps):
        s = first_sweep + k
        su2_heatbath_sweep(lat, beta, seed, s)
        if n_or:
            su2_overrelax(lat, n_or)
        if params is not None:
            su2_lp_forward(lat, params, lpwork, y)
            su2_lp_sweep(lat, beta, lp_seed, s, y, acc)
        su2_polyakov(lat, poly[k], with_corr=False)
        su2_plaquette(lat, plaq[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nx, ny, nz, nt = lat.n
    moves = n_sweeps * nx * ny * nz * nt
    return {
        "polyakov": poly[:, 0].cpu().tolist(),
        "plaquette": plaq[:, 0].cpu().tolist(),
        "acceptance": (acc.item() / moves) if params is not None else None,
        "wall_s": wall,
        "n_sweeps": n_sweeps,
    }


def thermalised_lattice(n, beta, seed, n_therm, prec="f64", device="cuda", n_or=0):
    lat = Lattice(n, prec, device=device)
    su2_init_hot(lat, seed)
    for s in range(n_therm):
        su2_heatbath_sweep(lat, beta, seed, s)
        if n_or:
            su2_overrelax(lat, n_or)
    return lat
