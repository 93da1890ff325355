"""The persistent batched sweep (su2_batch_sweep): one launch runs the heat
bath and n_or overrelaxation sweeps of every lattice of a batch, its blocks
meeting at a grid-wide barrier between classes.

- Bitwise the same links as the class launches (su2_batch_heatbath_sweep
  then su2_batch_overrelax), for a mixed batch (ragged shapes, plain and
  column addressing) and for the temperature scan's shapes, where every
  block takes many items of each class; n_or = 0 too.
- FP64 members match the oracle's heat-bath chain per link (1e-12).
- The barrier word's low 31 bits are 0 after every call.
- One captured launch (plus the sweep advance) per sweep replays bitwise
  like the eager class launches, replay after replay.
- A wait bounded by a tiny poll limit (forced from the host) gives up: the
  launch still ends, every lattice carries SU2_FLAG_SYNC, and the barrier
  word is left consistent.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 8, 4), (6, 4, 10, 8), (16, 16, 16, 4), (4, 6, 2, 12), (32, 16, 8, 2)]
BETAS = [2.2, 2.4, 2.6, 0.5, 2.7]
FLAG_SYNC = 4


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _sync():
    torch.cuda.synchronize()


def _lattices(su2, shapes, prec, seed):
    lats = []
    for j, n in enumerate(shapes):
        lat = su2.Lattice(n, prec, device="cuda", lattice_id=j)
        su2.su2_init_hot(lat, seed)
        lats.append(lat)
    return lats


def _flags(su2, lat):
    f = su2.su2_get_flags(lat)
    _sync()
    return int(f.item())


def _low_bits_clear(batch):
    return (int(batch.sync.item()) & 0x7FFFFFFF) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n_or", [2, 0])
def test_persistent_sweep_matches_class_launches(su2, prec, n_or):
    seed = 4242
    print(f"persistent sweep, mixed batch, {prec}, n_or {n_or}", flush=True)
    a = _lattices(su2, SHAPES, prec, seed)
    b = _lattices(su2, SHAPES, prec, seed)
    ba, bb = su2.Batch(a, BETAS), su2.Batch(b, BETAS)
    for s in range(3):
        su2.su2_batch_sweep(ba, seed, sweep=s, n_or=n_or)
        su2.su2_batch_heatbath_sweep(bb, seed, sweep=s)
        su2.su2_batch_overrelax(bb, n_or)
    _sync()
    assert _low_bits_clear(ba)
    for x, y in zip(a, b):
        assert torch.equal(x.links, y.links), x.n
        assert _flags(su2, x) == 0


def test_persistent_sweep_scan_shapes(su2):
    # 32^3x4, 48^3x6, 64^3x8 (the scan's shapes) with 4 overrelaxation
    # sweeps: 5648 items per class, several per block of the resident grid
    seed = 1234
    shapes = [(32, 32, 32, 4), (48, 48, 48, 6), (64, 64, 64, 8)]
    betas = [2.2, 2.4333, 2.6667]
    print("persistent sweep, scan shapes, f32, n_or 4", flush=True)
    a = _lattices(su2, shapes, "f32", seed)
    b = _lattices(su2, shapes, "f32", seed)
    ba, bb = su2.Batch(a, betas), su2.Batch(b, betas)
    for s in range(2):
        su2.su2_batch_sweep(ba, seed, sweep=s, n_or=4)
        su2.su2_batch_heatbath_sweep(bb, seed, sweep=s)
        su2.su2_batch_overrelax(bb, 4)
    _sync()
    assert _low_bits_clear(ba)
    for x, y in zip(a, b):
        assert torch.equal(x.links, y.links), x.n
        assert _flags(su2, x) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_persistent_sweep_graph_replay(su2, prec):
    seed, n_or, replays = 2025, 2, 4
    print(f"persistent sweep, graph replay, {prec}", flush=True)
    g = _lattices(su2, SHAPES, prec, seed)
    e = _lattices(su2, SHAPES, prec, seed)
    gb, eb = su2.Batch(g, BETAS), su2.Batch(e, BETAS)
    d_sweep = torch.zeros(1, dtype=torch.int32, device="cuda")
    _sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        su2.su2_batch_sweep(gb, seed, d_sweep=d_sweep, n_or=n_or)
        su2.su2_sweep_advance(d_sweep)
    _sync()
    assert int(d_sweep.item()) == 0
    for s in range(replays):
        graph.replay()
        su2.su2_batch_heatbath_sweep(eb, seed, sweep=s)
        su2.su2_batch_overrelax(eb, n_or)
        _sync()
        assert int(d_sweep.item()) == s + 1
        assert _low_bits_clear(gb)
        for x, y in zip(g, e):
            assert torch.equal(x.links, y.links), (s, x.n)


def test_persistent_sweep_gives_up_after_its_poll_limit(su2):
    # a poll limit of 1 makes nearly every barrier wait give up at once: the
    # launch must still end, flag every lattice, and leave the word's low
    # bits at 0 (each block still arrives once per barrier); a following
    # call with the default limit runs normally again
    seed = 99
    print("persistent sweep, poll limit 1", flush=True)
    lats = _lattices(su2, [(32, 32, 32, 4), (16, 16, 16, 4)], "f32", seed)
    batch = su2.Batch(lats, [2.3, 2.5])
    su2.su2_batch_sweep(batch, seed, sweep=0, n_or=2, spin_limit=1)
    _sync()
    assert _low_bits_clear(batch)
    for lat in lats:
        assert _flags(su2, lat) & FLAG_SYNC
    fresh = _lattices(su2, [(32, 32, 32, 4), (16, 16, 16, 4)], "f32", seed)
    ref = _lattices(su2, [(32, 32, 32, 4), (16, 16, 16, 4)], "f32", seed)
    fb, rb = su2.Batch(fresh, [2.3, 2.5]), su2.Batch(ref, [2.3, 2.5])
    fb.sync.copy_(batch.sync)                      # the word as the failed call left it
    su2.su2_batch_sweep(fb, seed, sweep=0, n_or=2)
    su2.su2_batch_heatbath_sweep(rb, seed, sweep=0)
    su2.su2_batch_overrelax(rb, 2)
    _sync()
    assert _low_bits_clear(fb)
    for x, y in zip(fresh, ref):
        assert torch.equal(x.links, y.links), x.n
        assert _flags(su2, x) == 0


def test_persistent_sweep_matches_oracle(su2):
    # FP64, two members of different shapes, couplings and lattice ids,
    # three persistent heat-bath sweeps (n_or = 0), per link against the
    # oracle chain of each
    seed = 1234
    shapes, betas, ids = [(8, 8, 8, 8), (6, 4, 10, 8)], [2.3, 2.5], [3, 9]
    print("persistent sweep against the oracle, f64", flush=True)
    lats = [su2.Lattice(n, "f64", device="cuda", lattice_id=i) for n, i in zip(shapes, ids)]
    refs = []
    for lat, n, i in zip(lats, shapes, ids):
        su2.su2_init_hot(lat, seed)
        refs.append(oracle.init_hot(n, seed, lattice_id=i))
    batch = su2.Batch(lats, betas)
    for s in range(3):
        su2.su2_batch_sweep(batch, seed, sweep=s, n_or=0)
        for ref, n, beta, i in zip(refs, shapes, betas, ids):
            assert oracle.heatbath_sweep(n, ref, beta, seed, s, lattice_id=i) == 0
        _sync()
        for lat, ref in zip(lats, refs):
            err = float(np.max(np.abs(su2.to_canonical(lat).numpy() - ref)))
            assert err <= 1e-12, (lat.n, s, err)
    assert _low_bits_clear(batch)
