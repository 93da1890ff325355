"""Benchmark: SU(2) link updates per second on one MI355X.

One step = one pass of the whole path on a resident lattice: 1 heat-bath
sweep (8 checkerboard launches) + 4 overrelaxation sweeps (32 launches) +
mean plaquette (taken by the last overrelaxation sweep from the staples it
forms, su2_overrelax_measured), Polyakov loop and its on-axis correlator
(su2_polyakov).  Default workload:
64^4 periodic lattice, beta = 2.3, FP32 links, hot start (Philox seed 1234).
The value counts 20 V link updates per step (4 V heat bath + 16 V
overrelaxation); the per-kernel roofline uses the algorithmic bytes of each
update (heat bath 8 links, overrelaxation 9 links of 16 B in FP32).

Prints ONE JSON line (rank 0).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
METRIC = "SU(2) link updates/sec + % HBM roofline; eff. indep. Polyakov samples/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--shape", type=str, default="64,64,64,64")
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--beta", type=float, default=2.3)
    ap.add_argument("--or-per-hb", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-shape", type=str, default=None,
                    help="lattice of the CPU-oracle sample (default: the benchmarked lattice)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum wall time of the CPU-oracle sample (whole steps)")
    ap.add_argument("--start", choices=["hot", "cold"], default="hot")
    ap.add_argument("--tile", type=int, default=0,
                    help="walk of the single lattice: 0 default strip, > 0 strip width, < 0 plain order")
    ap.add_argument("--tile-y", type=int, default=0,
                    help="row ranges per column in strip order (divides Ny; 0 default)")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="choose the walk with paper_1104_5432_amd.autotune before timing (untimed; "
                         "--no-autotune uses --tile/--tile-y)")
    ap.add_argument("--train", type=int, default=10000,
                    help="learned workload: heat-bath configurations to train on")
    ap.add_argument("--workload", choices=["single", "scan", "learned", "precision", "paper"], default="single",
                    help="single: one lattice (--shape); scan: 16 lattices mixing 32^3x4, 48^3x6, "
                         "64^3x8 at beta 2.2..2.7, one captured graph replay per sweep; learned: the "
                         "learned block proposal at 16^3x4; precision: FP32 against FP64 observables; "
                         "paper: the paper's own benchmark (random start, 100 heat-bath iterations at "
                         "beta 6.0 with the mean plaquette each) over lattice sizes, FP32 and FP64, "
                         "against one core of the CPU oracle")
    ap.add_argument("--persistent", action="store_true",
                    help="scan: run each sweep's heat bath and overrelaxation of all lattices in one "
                         "persistent launch (grid-wide barrier between classes) instead of one launch "
                         "per class")
    ap.add_argument("--fused-plaquette", action=argparse.BooleanOptionalAction, default=True,
                    help="take the plaquette in the last sweep of the step (no separate pass); "
                         "--no-fused-plaquette measures it with the one-pass measurement kernel")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of a plain device copy to run before the timed region "
                         "(reference for hardware byte counters)")
    return ap.parse_args()


# the sources of the global-memory update kernels, whose profiles give
# `traffic` (the LDS-staged kernels, other walks, have none)
SWEEP_SOURCES = ("su2_device.hpp", "su2_heatbath.hpp", "su2_kernels.hip", "su2_launch.hpp", "../build.py")


def csrc_sha256():
    """Hash of the sources of the sweep and observable kernels and of the
    build script (its flags), comments and blank lines left out, to tell
    whether a stored counter profile was taken from the current code."""
    import hashlib
    import re
    h = hashlib.sha256()
    try:
        for name in SWEEP_SOURCES:
            h.update(name.encode())
            with open(os.path.normpath(os.path.join(ROOT, "paper_1104_5432_amd", "csrc", name))) as f:
                text = f.read()
            comment = r"#[^\n]*" if name.endswith(".py") else r"//[^\n]*"
            code = [ln.rstrip() for ln in re.sub(comment, "", text).splitlines()]
            h.update("\n".join(ln for ln in code if ln).encode())
    except OSError:
        return None
    return h.hexdigest()


def profiled_traffic(kernel, prec, shape, walk):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE/WRITE_SIZE
    summaries under profiles/ (copy-calibrated), or None when no summary was
    taken from the current kernel sources with this lattice and walk."""
    import glob
    digest = csrc_sha256()
    if digest is None:
        return None
    want = {"kernel": kernel, "prec": prec, "shape": shape, "walk": "%d,%d" % tuple(walk), "csrc_sha256": digest}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                kv = dict(item.split("=", 1) for item in line.split()[1:])
                if all(kv.get(k) == v for k, v in want.items()):
                    return float(kv["bytes_per_launch"])
    return None


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(shape, beta, seed, n_or, min_seconds=10.0):
    """The FP64 CPU oracle timed on a bounded sample of the same workload:
    whole steps (1 heat-bath + n_or overrelaxation sweeps + plaquette +
    Polyakov loop/correlator) on the same lattice, repeated until at least
    min_seconds of wall time have been spent."""
    import oracle
    n = tuple(int(v) for v in shape.split(","))
    vol = n[0] * n[1] * n[2] * n[3]
    U = oracle.init_hot(n, seed)
    steps, dt = 0, 0.0
    while dt < min_seconds:
        t0 = time.perf_counter()
        oracle.heatbath_sweep(n, U, beta, seed, steps)
        for _ in range(n_or):
            oracle.overrelax_sweep(n, U)
        oracle.plaquette(n, U)
        oracle.polyakov_corr(n, U)
        dt += time.perf_counter() - t0
        steps += 1
    updates = 4 * vol * (1 + n_or) * steps
    return {
        "value": updates / dt,
        "unit": "link updates/s",
        "cores": oracle.num_threads(),
        "cpu": host_cpu_model(),
        "kind": "oracle",
        "sample": f"{'x'.join(map(str, n))} FP64 oracle, hot start, {steps} step(s) of 1 HB + {n_or} OR "
                  f"sweeps + plaquette + Polyakov/correlator, {dt:.1f} s wall",
    }


def scan(args):
    """Finite-temperature scan: 16 independent lattices, shapes cycling over
    32^3x4, 48^3x6, 64^3x8, beta_j = 2.2 + 0.5 j/15, lattice_id j, one
    captured graph per sweep (batched heat bath reading the sweep index from
    device memory, args.or_per_hb batched overrelaxation sweeps, Polyakov
    loop and correlator of all lattices in three launches, sweep advance).
    After the timed region the per-sweep correlators give each lattice's
    string tension (host analysis)."""
    import torch
    import paper_1104_5432_amd as su2

    shapes = [(32, 32, 32, 4), (48, 48, 48, 6), (64, 64, 64, 8)]
    lats, betas = [], []
    for j in range(16):
        lat = su2.Lattice(shapes[j % 3], args.prec, device="cuda:0", lattice_id=j)
        su2.su2_init_hot(lat, args.seed)
        lats.append(lat)
        betas.append(2.2 + 0.5 * j / 15)
    batch = su2.Batch(lats, betas)
    d_sweep = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    poly = torch.zeros((16, 2), dtype=torch.float64, device="cuda:0")
    corr = torch.zeros((16, max(min(lat.n[:3]) // 2 for lat in lats)), dtype=torch.float64, device="cuda:0")
    hist = torch.zeros((args.steps + args.warmup, 16, 2), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        if args.persistent:
            su2.su2_batch_sweep(batch, args.seed, d_sweep=d_sweep, n_or=args.or_per_hb)
        else:
            su2.su2_batch_heatbath_sweep(batch, args.seed, d_sweep=d_sweep)
            su2.su2_batch_overrelax(batch, args.or_per_hb)
        su2.su2_batch_polyakov(batch, poly, corr)
        su2.su2_sweep_advance(d_sweep)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    chist = torch.zeros((args.steps + args.warmup,) + tuple(corr.shape), dtype=torch.float64, device="cuda:0")

    def sweep(k):
        graph.replay()
        hist[k].copy_(poly, non_blocking=True)
        chist[k].copy_(corr, non_blocking=True)

    for k in range(args.warmup):
        sweep(k)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(args.steps):
        sweep(args.warmup + k)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    vol = sum(lat.volume for lat in lats)
    updates = 4 * vol * (1 + args.or_per_hb)
    flags = 0
    for lat in lats:
        flags |= int(su2.su2_get_flags(lat).item())
    absl = hist[args.warmup:, :, 0].abs().mean(0).cpu().tolist()
    sigma = scan_string_tension(lats, betas, chist[args.warmup:].cpu().numpy())
    rec = {
        "metric": METRIC,
        "value": updates * args.steps / (ms * 1e-3),
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": "finite-temperature scan: 16 SU(2) lattices cycling 32^3x4, 48^3x6, 64^3x8, "
                        "beta 2.2..2.7, hot start, per sweep one captured graph: 1 heat-bath + "
                        f"{args.or_per_hb} overrelaxation sweeps of all lattices "
                        + ("in one persistent launch " if args.persistent else "in one launch per class ")
                        + "+ Polyakov loop and correlator of each",
            "persistent": bool(args.persistent),
            "lattices": [list(lat.n) for lat in lats],
            "betas": betas,
            "link_updates_per_step": updates,
        },
        "polyakov_abs_mean_by_beta": dict(zip([round(b, 4) for b in betas], absl)),
        "string_tension_by_beta": sigma,
        "check": {"flags": flags},
    }
    print(json.dumps(rec), flush=True)


def scan_string_tension(lats, betas, corr_hist, n_blocks=20):
    """Host analysis of the scan's per-sweep correlators (eqs. (2)-(3) and
    the fit that follows them): for each lattice, a F(r) = -ln C(r)/Nt - ln 4/Nt
    fitted with a0 - a1/r + sigma r over r = 1..rmax, rmax the largest
    separation up to which every mean C(r) exceeds three of its standard
    errors (at least four points, else no fit); jackknife errors over blocks
    of consecutive sweeps (blocks shorter than the autocorrelation time make
    them optimistic)."""
    import numpy as np
    from paper_1104_5432_amd import analysis
    out = {}
    for j, (lat, beta) in enumerate(zip(lats, betas)):
        R = min(lat.n[:3]) // 2
        c = corr_hist[:, j, :R]
        if c.shape[0] < 2 * n_blocks:
            continue
        mean = c.mean(0)
        err = c.std(0, ddof=1) / np.sqrt(c.shape[0])
        ok = mean > 3 * err
        rmax = int(np.argmin(ok)) if not ok.all() else R
        if rmax < 4:
            out[round(beta, 4)] = {"nt": lat.n[3], "sigma": None, "rmax": rmax}
            continue
        p, perr, _ = analysis.string_tension(c, lat.n[3], rmin=1, rmax=rmax, n_blocks=n_blocks)
        out[round(beta, 4)] = {"nt": lat.n[3], "sigma": float(p[2]), "sigma_err": float(perr[2]), "rmax": rmax}
    return out


def learned_workload(args):
    """Learned proposal at 16^3 x 4, beta 2.30 (near deconfinement): train the
    network on args.train heat-bath configurations, then compare chains of
    args.steps sweeps -- heat bath; heat bath + 4 overrelaxation; heat bath +
    one learned sweep (trained, and untrained = mean-field coefficients) --
    by the integrated autocorrelation time of the Polyakov loop |L| and by
    effective independent samples per second, N / (2 tau_int) / wall time."""
    import torch
    from paper_1104_5432_amd import learned
    from paper_1104_5432_amd.stats import gamma_method

    n, beta, seed = (16, 16, 16, 4), 2.30, args.seed
    lat = learned.thermalised_lattice(n, beta, seed, 500, prec=args.prec)
    t0 = time.perf_counter()
    params, losses = learned.train(lat, beta, seed, args.train, first_sweep=500)
    t_train = time.perf_counter() - t0
    untrained = learned.init_params(seed)
    chains = {}
    for name, prm, n_or in (("heatbath", None, 0), ("heatbath+4or", None, 4),
                            ("heatbath+learned", params, 0), ("heatbath+untrained", untrained, 0),
                            ("heatbath+4or+learned", params, 4)):
        c = learned.thermalised_lattice(n, beta, seed + 7, 500, prec=args.prec)
        r = learned.run_chain(c, beta, seed + 7, args.steps, params=prm, n_or=n_or, first_sweep=500)
        absl = np.abs(np.array(r["polyakov"]))
        m, err, tau, win = gamma_method(absl)
        dtau = tau * np.sqrt(2.0 * (2 * win + 1) / args.steps)     # Wolff (2004), eq. (42)
        ms, es, taus, _ = gamma_method(np.array(r["polyakov"]))
        mp, ep, taup, _ = gamma_method(np.array(r["plaquette"]))
        chains[name] = {
            "tau_int_abs_polyakov": tau, "tau_int_abs_polyakov_err": dtau,
            "abs_polyakov": m, "abs_polyakov_err": err,
            "tau_int_polyakov": taus, "tau_int_plaquette": taup, "plaquette": mp, "plaquette_err": ep,
            "acceptance": r["acceptance"], "wall_s": r["wall_s"], "ms_per_sweep": 1e3 * r["wall_s"] / args.steps,
            "eff_samples_per_s": args.steps / (2 * tau) / r["wall_s"],
            "eff_samples_per_sweep": 1.0 / (2 * tau),
        }
        print(f"{name}: {chains[name]}", file=sys.stderr, flush=True)
    rec = {
        "metric": METRIC,
        "value": chains["heatbath+learned"]["eff_samples_per_s"],
        "unit": "eff. indep. Polyakov samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 500,
        "ms_per_step": chains["heatbath+learned"]["ms_per_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": "learned proposal: SU(2) 16^3x4, beta 2.30, hot start, network trained on "
                        f"{args.train} heat-bath configurations; chains of {args.steps} sweeps compared by "
                        "tau_int of |Polyakov loop|",
            "train_configs": args.train,
            "train_s": t_train,
            "loss_first_100": float(np.mean(losses[:100])),
            "loss_last_100": float(np.mean(losses[-100:])),
        },
        "chains": chains,
        "gain_vs_heatbath_per_s": chains["heatbath+learned"]["eff_samples_per_s"]
                                  / chains["heatbath"]["eff_samples_per_s"],
        "gain_vs_untrained_per_s": chains["heatbath+learned"]["eff_samples_per_s"]
                                   / chains["heatbath+untrained"]["eff_samples_per_s"],
    }
    print(json.dumps(rec), flush=True)


def oracle_one_core_rate(n, beta, seed, sweeps):
    """Link updates/s of the FP64 oracle on one host core (heat-bath sweeps
    with the plaquette after each), run in a child process whose OpenMP
    runtime is limited to one thread."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import oracle\n"
            "n = %r\nU = oracle.init_hot(n, %d)\nt = time.perf_counter()\n"
            "for s in range(%d):\n    oracle.heatbath_sweep(n, U, %r, %d, s); oracle.plaquette(n, U)\n"
            "dt = time.perf_counter() - t\nprint(oracle.num_threads(), dt)\n") % (ROOT, tuple(n), seed, sweeps, beta,
                                                                                seed)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    threads, dt = out.stdout.split()
    vol = n[0] * n[1] * n[2] * n[3]
    return 4 * vol * sweeps / float(dt), int(threads), float(dt)


def paper_workload(args):
    """The paper's own benchmark (Sec. 2.1): a random SU(2) start, then 100
    heat-bath iterations at beta = 6.0 with the mean plaquette computed at
    each, for several lattice sizes, in single and double precision, and
    the speed-up over one CPU core.  Here the plaquette is taken by each
    sweep's last classes (su2_heatbath_sweep_measured, a device array per
    iteration); each size is timed as a host loop of calls and as one
    captured graph of the 100 iterations (whose plaquettes must equal the
    loop's bitwise).  The CPU side is the FP64 oracle on one host core,
    timed on 20 iterations of a 16^4 lattice (its rate per link update does
    not depend on the size)."""
    import torch
    import paper_1104_5432_amd as su2
    from paper_1104_5432_amd import autotune

    beta, iters = 6.0, 100
    sizes = (8, 16, 24, 32, 48, 64)
    dev = torch.device("cuda:0")
    rows = []
    for prec in ("f32", "f64"):
        for L in sizes:
            n = (L, L, L, L)
            tile, tile_y = autotune.tune(n, prec, device=dev) if args.autotune else (0, 0)
            lat = su2.Lattice(n, prec, device=dev, tile=tile, tile_y=tile_y)
            plaq = torch.empty((iters, 7), dtype=torch.float64, device=dev)
            su2.su2_init_hot(lat, args.seed)
            for s in range(3):                                   # untimed warm-up
                su2.su2_heatbath_sweep(lat, beta, args.seed, s)
            su2.su2_init_hot(lat, args.seed)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for s in range(iters):
                su2.su2_heatbath_sweep_measured(lat, beta, args.seed, s, plaq[s])
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            # the same 100 iterations captured once in a graph and replayed from
            # the same start: the launches of small lattices stop waiting on the
            # host loop, and the plaquettes must come out bitwise the same
            eager = plaq.clone()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                for s in range(iters):
                    su2.su2_heatbath_sweep_measured(lat, beta, args.seed, s, plaq[s])
            su2.su2_init_hot(lat, args.seed)
            graph.replay()                                       # untimed: first replay uploads
            su2.su2_init_hot(lat, args.seed)
            torch.cuda.synchronize()
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ms_graph = e0.elapsed_time(e1)
            if not torch.equal(plaq, eager):
                raise RuntimeError(f"graph replay differs from the eager loop at {n} {prec}")
            vol = L ** 4
            rows.append({"lattice": list(n), "prec": prec, "ms_100_iterations": ms,
                         "link_updates_per_s": 4 * vol * iters / (ms * 1e-3),
                         "ms_100_iterations_graph": ms_graph,
                         "link_updates_per_s_graph": 4 * vol * iters / (ms_graph * 1e-3),
                         "plaquette_last": float(plaq[iters - 1, 0].item()), "walk": [tile, tile_y]})
            del lat, plaq, graph
            torch.cuda.empty_cache()
    cpu_rate, cpu_threads, cpu_s = oracle_one_core_rate((16, 16, 16, 16), beta, args.seed, 20)
    for r in rows:
        r["speedup_vs_one_core"] = r["link_updates_per_s"] / cpu_rate
        r["speedup_vs_one_core_graph"] = r["link_updates_per_s_graph"] / cpu_rate
    head = next(r for r in rows if r["prec"] == "f32" and r["lattice"][0] == 64)
    rec = {
        "metric": METRIC,
        "value": head["link_updates_per_s"],
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": 3,
        "ms_per_step": head["ms_100_iterations"] / iters,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "the paper's benchmark: random SU(2) start, 100 heat-bath iterations at beta 6.0 with "
                        "the mean plaquette each, lattices 8^4..64^4, FP32 and FP64; value: 64^4 FP32",
        },
        "by_size": rows,
        "cpu_one_core": {"value": cpu_rate, "unit": "link updates/s", "cores": cpu_threads, "cpu": host_cpu_model(),
                         "kind": "oracle",
                         "sample": f"16^4 FP64 oracle, 20 heat-bath iterations with the plaquette, {cpu_s:.1f} s"},
    }
    print(json.dumps(rec), flush=True)


def precision_workload(args):
    """FP32 against FP64 links on the benchmarked lattice: for beta 2.3, 2.5
    and 6.0 an FP64 and an FP32 chain (hot start, args.steps steps of 1 heat
    bath + args.or_per_hb overrelaxation sweeps), and for every observable the
    plaquette and the Polyakov-loop calls return -- the mean plaquette and its
    six planes, the signed mean L, |mean L|, the mean of |L(x)| and the
    correlator C(r) at every r -- the difference of the two chains' means in
    units of the combined Gamma-method error, after discarding the first 20%
    of the steps."""
    import torch
    import paper_1104_5432_amd as su2
    from paper_1104_5432_amd.stats import gamma_method

    n = tuple(int(v) for v in args.shape.split(","))
    rmax = min(n[:3]) // 2
    dev = torch.device("cuda:0")
    rows = {}
    t0 = time.perf_counter()
    planes = ("01", "02", "03", "12", "13", "23")
    for beta in (2.3, 2.5, 6.0):
        res = {}
        for prec in ("f64", "f32"):
            lat = su2.Lattice(n, prec, device=dev)
            su2.su2_init_hot(lat, args.seed)
            plaq = torch.empty((args.steps, 7), dtype=torch.float64, device=dev)
            poly = torch.empty((args.steps, 2), dtype=torch.float64, device=dev)
            corr = torch.empty((args.steps, rmax), dtype=torch.float64, device=dev)
            for s in range(args.steps):
                su2.su2_heatbath_sweep(lat, beta, args.seed, s)
                su2.su2_overrelax(lat, args.or_per_hb)
                su2.su2_plaquette(lat, plaq[s])
                su2.su2_polyakov(lat, poly[s], corr[s])
            torch.cuda.synchronize()
            cut = args.steps // 5
            P, L, C = (t[cut:].cpu().numpy() for t in (plaq, poly, corr))
            series = {"plaquette": P[:, 0], "polyakov": L[:, 0], "abs_polyakov": np.abs(L[:, 0]),
                      "mean_abs_L": L[:, 1]}
            for j, name in enumerate(planes):
                series["plane_" + name] = P[:, 1 + j]
            for r in range(1, rmax + 1):
                series[f"corr_r{r}"] = C[:, r - 1]
            res[prec] = {k: gamma_method(v)[:2] for k, v in series.items()}
            res[prec]["flags"] = int(su2.su2_get_flags(lat).item())
            del lat
        row = {}
        for obs in res["f64"]:
            if obs == "flags":
                continue
            (m64, e64), (m32, e32) = res["f64"][obs], res["f32"][obs]
            err = float(np.hypot(e64, e32))
            row[obs] = {"f64": m64, "f64_err": e64, "f32": m32, "f32_err": e32, "diff": m32 - m64,
                        "z": (m32 - m64) / err if err > 0 else 0.0}
        row["flags"] = res["f64"]["flags"] | res["f32"]["flags"]
        rows[str(beta)] = row
        zs = {k: v["z"] for k, v in row.items() if k != "flags"}
        worst = max(zs, key=lambda k: abs(zs[k]))
        print(f"beta {beta}: {len(zs)} observables, max |z| {abs(zs[worst]):.2f} ({worst}); "
              f"plaquette diff {row['plaquette']['diff']:+.2e} z {row['plaquette']['z']:+.2f}; "
              f"|L| diff {row['abs_polyakov']['diff']:+.2e} z {row['abs_polyakov']['z']:+.2f}; "
              f"flags {row['flags']}", file=sys.stderr, flush=True)
    zmax = max(abs(v["z"]) for r in rows.values() for k, v in r.items() if k != "flags")
    nobs = sum(1 for r in rows.values() for k in r if k != "flags")
    rec = {
        "metric": "FP32 - FP64 observable difference (max |z| over beta and observables)",
        "value": zmax,
        "unit": "combined standard errors",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.steps // 5,
        "ms_per_step": 1e3 * (time.perf_counter() - t0) / (6 * args.steps),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 vs f64",
        "data": "synthetic",
        "config": {
            "workload": f"SU(2) {'x'.join(map(str, n))}, hot start (Philox seed {args.seed}), FP32 and FP64 "
                        f"chains of {args.steps} steps of 1 heat-bath + {args.or_per_hb} overrelaxation sweeps "
                        "at beta 2.3, 2.5, 6.0; every observable of the plaquette and Polyakov-loop calls "
                        "(mean plaquette, six planes, signed mean L, |mean L|, mean |L(x)|, C(r) for every r), "
                        "Gamma-method errors",
            "lattice": list(n),
            "observables_compared": nobs,
        },
        "by_beta": rows,
    }
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(one lattice is updated on one GPU; sharding is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "scan":
        scan(args)
        return
    if args.workload == "learned":
        learned_workload(args)
        return
    if args.workload == "precision":
        precision_workload(args)
        return
    if args.workload == "paper":
        paper_workload(args)
        return

    import torch
    import paper_1104_5432_amd as su2

    n = tuple(int(v) for v in args.shape.split(","))
    vol = n[0] * n[1] * n[2] * n[3]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    tile, tile_y = args.tile, args.tile_y
    if args.autotune and not (args.tile or args.tile_y):
        from paper_1104_5432_amd import autotune
        tile, tile_y = autotune.tune(n, args.prec, device=dev)
    lat = su2.Lattice(n, args.prec, device=dev, tile=tile, tile_y=tile_y)
    if args.start == "hot":
        su2.su2_init_hot(lat, args.seed)
    else:
        su2.su2_init_cold(lat)
    plaq = torch.empty((max(args.steps, 1), 7), dtype=torch.float64, device=dev)
    poly = torch.empty((max(args.steps, 1), 2), dtype=torch.float64, device=dev)
    corr = torch.empty((max(args.steps, 1), max(1, min(n[:3]) // 2)), dtype=torch.float64, device=dev)

    if args.calibrate_copy:
        a = torch.empty(args.calibrate_copy, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # With the fused plaquette the last sweep of the step measures it and
    # the Polyakov pass follows; the overrelaxation events bracket only the
    # plain sweeps before that last one (the kernel the roofline reports),
    # unless the step has a single overrelaxation sweep.
    fused = args.fused_plaquette
    or_plain = args.or_per_hb - 1 if fused and args.or_per_hb >= 2 else args.or_per_hb

    def step(s, ev=None):
        k = s - args.warmup if s >= args.warmup else 0
        if ev:
            ev[0].record(stream)
        if fused and args.or_per_hb == 0:
            su2.su2_heatbath_sweep_measured(lat, args.beta, args.seed, s, plaq[k])
        else:
            su2.su2_heatbath_sweep(lat, args.beta, args.seed, s)
        if ev:
            ev[1].record(stream)
        if fused and args.or_per_hb == 1:
            su2.su2_overrelax_measured(lat, 1, plaq[k])
        elif or_plain:
            su2.su2_overrelax(lat, or_plain)
        if ev:
            ev[2].record(stream)
        if not fused:
            su2.su2_measure(lat, plaq[k], poly[k], corr[k])     # plaquette, Polyakov loop, correlator
            return
        if args.or_per_hb >= 2:
            su2.su2_overrelax_measured(lat, 1, plaq[k])
        su2.su2_polyakov(lat, poly[k], corr[k])

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for i in range(args.steps):
        step(args.warmup + i, evs[i])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    hb_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    or_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps

    flags = int(su2.su2_get_flags(lat).item())
    last_plaq = float(plaq[args.steps - 1, 0].item())
    last_poly = float(poly[args.steps - 1, 1].item())

    link_b = 16 if args.prec == "f32" else 32
    half = vol // 2
    or_launch_ms = or_ms / (8 * or_plain) if or_plain else float("nan")
    hb_launch_ms = hb_ms / 8
    or_bytes = half * 9 * link_b          # algorithmic bytes per overrelaxation launch
    hb_bytes = half * 8 * link_b          # algorithmic bytes per heat-bath launch
    or_gbs = or_bytes / (or_launch_ms * 1e-3) / 1e9 if args.or_per_hb else float("nan")
    hb_gbs = hb_bytes / (hb_launch_ms * 1e-3) / 1e9
    updates = 4 * vol * (1 + args.or_per_hb)
    value = updates * args.steps / (ms_total * 1e-3)

    or_roof = {
        "kernel": "overrelax_kernel",
        "achieved": or_gbs,
        "frac": or_gbs / HBM_PEAK_GBS,
        "traffic": profiled_traffic("overrelax_kernel", args.prec, args.shape, (tile, tile_y)),
        "bytes_per_launch": or_bytes,
        "avg_launch_ms": or_launch_ms,
    }
    hb_roof = {
        "kernel": "heatbath_kernel",
        "achieved": hb_gbs,
        "frac": hb_gbs / HBM_PEAK_GBS,
        "traffic": profiled_traffic("heatbath_kernel", args.prec, args.shape, (tile, tile_y)),
        "bytes_per_launch": hb_bytes,
        "avg_launch_ms": hb_launch_ms,
    }
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": f"SU(2) pure gauge {'^'.join([str(n[0]), '4']) if len(set(n)) == 1 else 'x'.join(map(str, n))} "
                        f"periodic, beta={args.beta}, {args.start} start (Philox seed {args.seed}), "
                        f"{args.prec.upper()} links, per step 1 heat-bath + {args.or_per_hb} overrelaxation "
                        f"sweeps + FP64 plaquette ({'taken by the last sweep' if fused else 'measurement pass'}) "
                        f"+ Polyakov loop/correlator",
            "lattice": list(n),
            "beta": args.beta,
            "or_per_hb": args.or_per_hb,
            "tile": tile,
            "tile_y": tile_y,
            "start": args.start,
            "fused_plaquette": fused,
            "link_updates_per_step": updates,
        },
        # the dominant kernel: overrelaxation when the step has any, else heat bath
        "roofline": dict(or_roof if args.or_per_hb else hb_roof, bound="hbm", peak=HBM_PEAK_GBS, unit="GB/s"),
        "heatbath_roofline": hb_roof,
        "overrelax_roofline": or_roof if args.or_per_hb else None,
        "sweep_roofline_frac": ((hb_bytes * 8 + or_bytes * 8 * or_plain) / ((hb_ms + or_ms) * 1e-3) / 1e9)
                               / HBM_PEAK_GBS,
        "wall_s_timed": wall,
        "check": {"plaquette_last": last_plaq, "polyakov_abs_last": last_poly, "flags": flags},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args.cpu_shape or args.shape, args.beta, args.seed, args.or_per_hb,
                                           args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
