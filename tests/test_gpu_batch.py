"""Batched lattices (a temperature scan in one launch per class) and
captured-graph replay, through the C ABI.

- A lattice updated inside a batch gives bit-identical links to the same
  lattice (same lattice_id, seed, beta) updated alone: the random numbers are
  keyed by (seed, sweep, site, mu, kind, lattice_id) and the update of a link
  does not depend on which block or launch performs it -- also for the
  large lattices whose overrelaxation runs as launches of their own.
- Batch members match the FP64 oracle per link (same bound as single runs).
- The batched Polyakov loop and correlator are bitwise the per-lattice
  ones and leave the correlator rows beyond each lattice's range untouched.
- A hipGraph capturing one sweep (batched heat bath with the sweep index read
  from device memory, batched overrelaxation, observables, sweep advance)
  replays bit-identically to the same calls made eagerly, replay after
  replay, with eager work and synchronisations in between.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 8, 4), (6, 4, 10, 8), (16, 16, 16, 4), (4, 6, 2, 12), (32, 16, 8, 2)]
BETAS = [2.2, 2.4, 2.6, 0.5, 2.7]


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _sync():
    torch.cuda.synchronize()


def _fresh(su2, prec, seed, tiles=None):
    lats = []
    for j, n in enumerate(SHAPES):
        lat = su2.Lattice(n, prec, device="cuda", lattice_id=j, tile=0 if tiles is None else tiles[j])
        su2.su2_init_hot(lat, seed)
        lats.append(lat)
    return lats


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_single_lattices(su2, prec):
    seed = 77
    batched = _fresh(su2, prec, seed)
    single = _fresh(su2, prec, seed, tiles=[-1, 1, 2, -1, 4])   # other walks, same results
    batch = su2.Batch(batched, BETAS)
    for s in range(3):
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=s)
        su2.su2_batch_overrelax(batch, 2)
        for lat, beta in zip(single, BETAS):
            su2.su2_heatbath_sweep(lat, beta, seed, s)
            su2.su2_overrelax(lat, 2)
    _sync()
    for a, b in zip(batched, single):
        assert torch.equal(a.links, b.links), a.n
        f = su2.su2_get_flags(a)
        _sync()
        assert int(f.item()) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_with_own_launch_lattices_matches_single_lattices(su2, prec):
    # lattices of >= 2^20 sites run their overrelaxation classes as launches
    # of their own (the capped single-lattice kernel), the others in the
    # batched launch, whose table leaves them an empty range: large lattices
    # first, between small ones and last, bitwise as each lattice alone
    seed = 79
    shapes = [(64, 64, 32, 8), (8, 8, 8, 4), (32, 32, 32, 32), (16, 16, 16, 4), (6, 4, 10, 8), (64, 64, 64, 4)]
    betas = [2.3, 2.2, 2.5, 2.6, 0.5, 2.4]
    print(f"batch with own-launch lattices, {prec}", flush=True)

    def fresh():
        out = []
        for j, n in enumerate(shapes):
            lat = su2.Lattice(n, prec, device="cuda", lattice_id=j)
            su2.su2_init_hot(lat, seed)
            out.append(lat)
        return out

    batched, single = fresh(), fresh()
    assert sum(int(np.prod(n)) >= 1 << 20 for n in shapes) == 3
    batch = su2.Batch(batched, betas)
    for s in range(2):
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=s)
        su2.su2_batch_overrelax(batch, 2)
        for lat, beta in zip(single, betas):
            su2.su2_heatbath_sweep(lat, beta, seed, s)
            su2.su2_overrelax(lat, 2)
    _sync()
    for a, b in zip(batched, single):
        assert torch.equal(a.links, b.links), a.n
        f = su2.su2_get_flags(a)
        _sync()
        assert int(f.item()) == 0


def test_graph_replay_with_own_launch_lattices(su2):
    # the large lattices' own overrelaxation launches inside a captured
    # graph replay like the same calls made eagerly, replay after replay
    seed, n_or, replays = 83, 2, 3
    shapes = [(8, 8, 8, 4), (64, 64, 32, 8), (16, 16, 16, 4), (32, 32, 32, 32)]
    betas = [2.2, 2.3, 2.6, 2.5]
    print("graph replay with own-launch lattices", flush=True)

    def fresh():
        out = []
        for j, n in enumerate(shapes):
            lat = su2.Lattice(n, "f32", device="cuda", lattice_id=j)
            su2.su2_init_hot(lat, seed)
            out.append(lat)
        return out

    g_lats, e_lats = fresh(), fresh()
    g_batch, e_batch = su2.Batch(g_lats, betas), su2.Batch(e_lats, betas)
    d_sweep = torch.zeros(1, dtype=torch.int32, device="cuda")
    _sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        su2.su2_batch_heatbath_sweep(g_batch, seed, d_sweep=d_sweep)
        su2.su2_batch_overrelax(g_batch, n_or)
        su2.su2_sweep_advance(d_sweep)
    _sync()
    assert int(d_sweep.item()) == 0
    for s in range(replays):
        graph.replay()
        su2.su2_batch_heatbath_sweep(e_batch, seed, sweep=s)
        su2.su2_batch_overrelax(e_batch, n_or)
        _sync()
        assert int(d_sweep.item()) == s + 1
        for a, b in zip(g_lats, e_lats):
            assert torch.equal(a.links, b.links), (s, a.n)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_polyakov_matches_single_lattices(su2, prec):
    # su2_batch_polyakov: three launches for all lattices, bitwise the
    # per-lattice su2_polyakov (same partials, same summation order)
    seed = 91
    lats = _fresh(su2, prec, seed)
    batch = su2.Batch(lats, BETAS)
    for s in range(2):
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=s)
        su2.su2_batch_overrelax(batch, 1)
    stride = 11                                    # wider than any min(Nx,Ny,Nz)/2 here
    sentinel = -7.25
    corr = torch.full((len(lats), stride), sentinel, dtype=torch.float64, device="cuda")
    poly, corr = su2.su2_batch_polyakov(batch, corr=corr)
    poly_nc, none = su2.su2_batch_polyakov(batch, with_corr=False)
    _sync()
    assert none is None
    assert torch.equal(poly, poly_nc)
    for j, lat in enumerate(lats):
        q, c = su2.su2_polyakov(lat)
        _sync()
        r = min(lat.n[:3]) // 2
        assert torch.equal(poly[j], q), lat.n
        assert torch.equal(corr[j, :r], c[:r]), lat.n
        assert torch.all(corr[j, r:] == sentinel), lat.n      # left untouched beyond rmax
    # against the oracle on the links the GPU holds
    for j in (0, 3):
        Uc = su2.to_canonical(lats[j]).numpy()
        n = lats[j].n
        l_mean, l_abs = oracle.polyakov(n, Uc)
        C = oracle.polyakov_corr(n, Uc)
        tol = 1e-13 if prec == "f64" else 2e-6
        g = poly[j].cpu().numpy()
        assert abs(g[0] - l_mean) <= tol and abs(g[1] - l_abs) <= tol
        assert np.max(np.abs(corr[j, :len(C)].cpu().numpy() - C)) <= tol


def test_batch_members_match_oracle(su2):
    seed = 1234
    shapes = [(8, 8, 8, 8), (6, 4, 10, 8)]
    betas = [2.3, 2.5]
    ids = [2, 5]
    lats = [su2.Lattice(n, "f64", device="cuda", lattice_id=i) for n, i in zip(shapes, ids)]
    refs = []
    for lat, n, i in zip(lats, shapes, ids):
        su2.su2_init_hot(lat, seed)
        refs.append(oracle.init_hot(n, seed, lattice_id=i))
    batch = su2.Batch(lats, betas)
    for s in range(3):
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=s)
        for ref, n, beta, i in zip(refs, shapes, betas, ids):
            oracle.heatbath_sweep(n, ref, beta, seed, s, lattice_id=i)
        _sync()
        for lat, ref in zip(lats, refs):
            err = float(np.max(np.abs(su2.to_canonical(lat).numpy() - ref)))
            assert err <= 1e-12, (lat.n, s, err)


def test_batch_scan_shapes_match_oracle(su2):
    # The temperature scan's three shapes (32^3x4, 48^3x6, 64^3x8) as scan
    # members j = 0, 7, 14 (shape j mod 3, beta_j = 2.2 + 0.5 j / 15,
    # lattice_id j), FP64, in one batch: one heat-bath sweep and one
    # overrelaxation sweep, per link against the oracle chain of each.
    seed = 1234
    members = (0, 7, 14)
    scan_shapes = [(32, 32, 32, 4), (48, 48, 48, 6), (64, 64, 64, 8)]
    shapes = [scan_shapes[j % 3] for j in members]
    betas = [2.2 + 0.5 * j / 15 for j in members]
    print("batched scan shapes", shapes, "betas", [round(b, 4) for b in betas], flush=True)
    lats = [su2.Lattice(n, "f64", device="cuda", lattice_id=j) for n, j in zip(shapes, members)]
    for lat in lats:
        su2.su2_init_hot(lat, seed)
    batch = su2.Batch(lats, betas)
    su2.su2_batch_heatbath_sweep(batch, seed, sweep=0)
    su2.su2_batch_overrelax(batch, 1)
    _sync()
    for lat, n, beta, j in zip(lats, shapes, betas, members):
        ref = oracle.init_hot(n, seed, lattice_id=j)
        assert oracle.heatbath_sweep(n, ref, beta, seed, 0, lattice_id=j) == 0
        oracle.overrelax_sweep(n, ref)
        err = float(np.max(np.abs(su2.to_canonical(lat).numpy() - ref)))
        print(f"  {n} beta {beta:.4f} id {j}: max |dU| = {err:.2e}", flush=True)
        assert err <= 1e-12, (n, err)
        f = su2.su2_get_flags(lat)
        _sync()
        assert int(f.item()) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replay_matches_eager(su2, prec):
    seed, n_or, replays = 2024, 2, 5
    g_lats = _fresh(su2, prec, seed)
    e_lats = _fresh(su2, prec, seed)
    g_batch, e_batch = su2.Batch(g_lats, BETAS), su2.Batch(e_lats, BETAS)
    d_sweep = torch.zeros(1, dtype=torch.int32, device="cuda")
    plaq = [torch.zeros(7, dtype=torch.float64, device="cuda") for _ in g_lats]
    poly = [torch.zeros(2, dtype=torch.float64, device="cuda") for _ in g_lats]
    corr = [torch.zeros(max(1, min(l.n[:3]) // 2), dtype=torch.float64, device="cuda") for l in g_lats]
    _sync()

    bpoly = torch.zeros((len(g_lats), 2), dtype=torch.float64, device="cuda")
    bcorr = torch.zeros((len(g_lats), max(c.numel() for c in corr)), dtype=torch.float64, device="cuda")
    _sync()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        su2.su2_batch_heatbath_sweep(g_batch, seed, d_sweep=d_sweep)
        su2.su2_batch_overrelax(g_batch, n_or)
        for lat, p, q, c in zip(g_lats, plaq, poly, corr):
            su2.su2_plaquette(lat, p)
            su2.su2_polyakov(lat, q, c)
        su2.su2_batch_polyakov(g_batch, bpoly, bcorr)
        su2.su2_sweep_advance(d_sweep)
    _sync()
    # capturing must not have executed anything
    assert int(d_sweep.item()) == 0

    for s in range(replays):
        graph.replay()
        # eager reference, with its own synchronisations in between
        su2.su2_batch_heatbath_sweep(e_batch, seed, sweep=s)
        su2.su2_batch_overrelax(e_batch, n_or)
        _sync()
        assert int(d_sweep.item()) == s + 1
        for lat_g, lat_e, p, q, c in zip(g_lats, e_lats, plaq, poly, corr):
            assert torch.equal(lat_g.links, lat_e.links), (s, lat_g.n)
            pe = su2.su2_plaquette(lat_e)
            qe, ce = su2.su2_polyakov(lat_e)
            _sync()
            assert torch.equal(p, pe) and torch.equal(q, qe) and torch.equal(c[:len(ce)], ce), (s, lat_g.n)
        for j, (q, c) in enumerate(zip(poly, corr)):
            assert torch.equal(bpoly[j], q) and torch.equal(bcorr[j, :c.numel()], c), (s, j)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replay_of_the_measured_step(su2, prec):
    # the benchmark's step in a captured graph: heat bath (a batch of one,
    # sweep index from device memory), overrelaxation whose last sweep takes
    # the plaquette, Polyakov loop and correlator; every replay equals the
    # same calls made eagerly, with eager work and synchronisations between
    seed, n = 808, (8, 8, 8, 4)
    g_lat = su2.Lattice(n, prec, device="cuda", lattice_id=3)
    e_lat = su2.Lattice(n, prec, device="cuda", lattice_id=3)
    for lat in (g_lat, e_lat):
        su2.su2_init_hot(lat, seed)
    g_batch = su2.Batch([g_lat], [2.4])
    d_sweep = torch.zeros(1, dtype=torch.int32, device="cuda")
    plaq = torch.zeros(7, dtype=torch.float64, device="cuda")
    poly = torch.zeros(2, dtype=torch.float64, device="cuda")
    corr = torch.zeros(min(n[:3]) // 2, dtype=torch.float64, device="cuda")
    _sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        su2.su2_batch_heatbath_sweep(g_batch, seed, d_sweep=d_sweep)
        su2.su2_overrelax_measured(g_lat, 3, plaq)
        su2.su2_polyakov(g_lat, poly, corr)
        su2.su2_sweep_advance(d_sweep)
    _sync()
    for s in range(4):
        graph.replay()
        su2.su2_heatbath_sweep(e_lat, 2.4, seed, s)
        pe = su2.su2_overrelax_measured(e_lat, 3)
        qe, ce = su2.su2_polyakov(e_lat)
        _sync()
        assert torch.equal(g_lat.links, e_lat.links), s
        assert torch.equal(plaq, pe) and torch.equal(poly, qe) and torch.equal(corr, ce), s


def test_many_lattice_batch_matches_single_lattices(su2):
    # 130 lattices: the block -> lattice lookup takes three rounds of wave
    # ballots (64 entries each); tiny and ragged shapes, one block each
    shapes = [(2, 2, 2, 2), (4, 2, 2, 2), (2, 4, 6, 2), (4, 4, 4, 4)]
    seed, count = 55, 130
    batched, single, betas = [], [], []
    for j in range(count):
        n = shapes[j % len(shapes)]
        for group in (batched, single):
            lat = su2.Lattice(n, "f32", device="cuda", lattice_id=j)
            su2.su2_init_hot(lat, seed)
            group.append(lat)
        betas.append(1.5 + j / count)
    batch = su2.Batch(batched, betas)
    for s in range(2):
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=s)
        su2.su2_batch_overrelax(batch, 1)
        for lat, beta in zip(single, betas):
            su2.su2_heatbath_sweep(lat, beta, seed, s)
            su2.su2_overrelax(lat, 1)
    poly, corr = su2.su2_batch_polyakov(batch)
    _sync()
    for j, (a, b) in enumerate(zip(batched, single)):
        assert torch.equal(a.links, b.links), j
        q, c = su2.su2_polyakov(b)
        _sync()
        assert torch.equal(poly[j], q) and torch.equal(corr[j, :c.numel()], c), j
