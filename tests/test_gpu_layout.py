"""The skewed FP64 link layout on the GPU.  A lattice with V/2 >= 2^18 keeps
its 16 sub-planes V/2 + 16392 elements apart; every kernel family must
address them at that stride and never touch the skew elements between
them.  Two copies of one lattice, one with NaN in every skew element and
one with zeros, go through the same calls -- single-lattice updates on the
strip, plain and LDS-staged walks, the sweeps and passes that take the
plaquette and Polyakov loop, the batched and persistent sweeps, the learned
block move -- and must give bitwise the same links and observables, with
the NaN left where it was.  A skewed lattice of a shape that takes the
kernels' coordinate addressing matches the oracle class by class."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N = (64, 64, 16, 8)  # V/2 = 2^18, the smallest skewed volume
HALF = 64 * 64 * 16 * 8 // 2


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _sub_planes(su2, lat):
    S = su2.su2_plane_stride(lat.n, "f64")
    assert S == HALF + 16392
    return lat.links.view(torch.float64).view(16, S, 2)


def _pair(su2, seed, tile=0, lattice_id=0):
    a = su2.Lattice(N, "f64", device="cuda", tile=tile, lattice_id=lattice_id)
    b = su2.Lattice(N, "f64", device="cuda", tile=tile, lattice_id=lattice_id)
    for lat in (a, b):
        su2.su2_init_hot(lat, seed)
    _sub_planes(su2, a)[:, HALF:].fill_(float("nan"))
    _sub_planes(su2, b)[:, HALF:].zero_()
    return a, b


def _same(su2, a, b):
    torch.cuda.synchronize()
    pa, pb = _sub_planes(su2, a), _sub_planes(su2, b)
    assert torch.equal(pa[:, :HALF], pb[:, :HALF])
    assert not torch.isnan(pa[:, :HALF]).any()
    assert torch.isnan(pa[:, HALF:]).all()
    assert (pb[:, HALF:] == 0).all()


def _flags_clear(su2, *lats):
    for lat in lats:
        f = su2.su2_get_flags(lat)
        torch.cuda.synchronize()
        assert int(f.item()) == 0


@pytest.mark.parametrize("tile", [0, -1, -3])
def test_skew_untouched_by_single_lattice_calls(su2, tile):
    print(f"skewed FP64 layout, single-lattice calls, tile {tile}", flush=True)
    seed = 808
    a, b = _pair(su2, seed, tile)
    _same(su2, a, b)
    out = []
    for lat in (a, b):
        su2.su2_heatbath_sweep(lat, 2.3, seed, 0)
        su2.su2_overrelax(lat, 2)
        r = [su2.su2_heatbath_sweep_measured(lat, 2.3, seed, 1), su2.su2_overrelax_measured(lat, 1),
             su2.su2_plaquette(lat)]
        r += list(su2.su2_polyakov(lat))
        r += list(su2.su2_measure(lat))
        out.append(r)
    _same(su2, a, b)
    for x, y in zip(*out):
        assert torch.equal(x, y)
    _flags_clear(su2, a, b)


def test_skew_untouched_by_batched_and_persistent_sweeps(su2):
    print("skewed FP64 layout, batched and persistent sweeps", flush=True)
    seed = 809
    a, b = _pair(su2, seed, lattice_id=3)
    c, d = _pair(su2, seed + 1, lattice_id=4)
    out = []
    for lats in ((a, c), (b, d)):
        batch = su2.Batch(list(lats), [2.3, 2.5])
        su2.su2_batch_heatbath_sweep(batch, seed, sweep=0)
        su2.su2_batch_overrelax(batch, 2)
        su2.su2_batch_sweep(batch, seed, sweep=1, n_or=2)
        out.append(su2.su2_batch_polyakov(batch))
    _same(su2, a, b)
    _same(su2, c, d)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    _flags_clear(su2, a, b, c, d)


def test_skew_untouched_by_learned_block_move(su2):
    print("skewed FP64 layout, learned block move", flush=True)
    seed = 810
    a, b = _pair(su2, seed)
    g = torch.Generator(device="cpu").manual_seed(5)
    y = (0.1 * torch.randn(HALF * 2 * 6, generator=g)).to(torch.float32).cuda()
    acc = []
    for lat in (a, b):
        n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
        su2.su2_lp_sweep(lat, 2.3, seed, 0, y, n_acc)
        acc.append(n_acc)
    _same(su2, a, b)
    assert torch.equal(acc[0], acc[1]) and int(acc[0].item()) > 0
    _flags_clear(su2, a, b)


@pytest.mark.parametrize("mu,par", [(0, 1), (3, 0)])
def test_skewed_lattice_of_unaligned_shape_matches_oracle(su2, mu, par):
    # 70 x 62 x 16 x 8: V/2 = 277760 (skewed) and columns of 2170 checkerboard
    # sites, not a multiple of a wave, so the kernels take the coordinate
    # path; one heat-bath class and one overrelaxation class per link
    # against the oracle
    import numpy as np
    import oracle
    n = (70, 62, 16, 8)
    half = 70 * 62 * 16 * 8 // 2
    assert su2.su2_plane_stride(n, "f64") == half + 16392
    print(f"skewed FP64 layout, {n}, class ({mu},{par}) against the oracle", flush=True)
    seed, beta = 515, 2.3
    U = oracle.init_hot(n, seed)
    lat = su2.Lattice(n, "f64", device="cuda")
    su2.from_canonical(lat, U)
    assert oracle.heatbath_halfsweep(n, U, beta, seed, 3, mu, par) == 0
    su2.su2_heatbath_halfsweep(lat, beta, seed, 3, mu, par)
    torch.cuda.synchronize()
    assert np.max(np.abs(su2.to_canonical(lat).numpy() - U)) <= 1e-13
    oracle.overrelax_halfsweep(n, U, (mu + 1) % 4, 1 - par)
    su2.su2_overrelax_halfsweep(lat, (mu + 1) % 4, 1 - par)
    torch.cuda.synchronize()
    assert np.max(np.abs(su2.to_canonical(lat).numpy() - U)) <= 1e-13
    _flags_clear(su2, lat)
