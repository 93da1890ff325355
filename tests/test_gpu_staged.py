"""The LDS-staged updates (walk tile = -2: overrelaxation; -3: heat bath
too) against the global-memory kernels: the staple is formed from the LDS
copies with the same products and sums in the same order, and the heat
bath samples with the same random words and arithmetic, so every class
must give bitwise the same links, in both precisions, on small lattices
(slabs with wrapped halos, several slice chunks) and on the benchmarked
64^4."""
import pytest

import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _pair(su2, n, prec, seed, tile=-2):
    staged = su2.Lattice(n, prec, device="cuda", tile=tile)
    plain = su2.Lattice(n, prec, device="cuda")
    su2.su2_init_hot(plain, seed)
    su2.su2_heatbath_sweep(plain, 2.3, seed, 0)
    staged.links.copy_(plain.links)
    return staged, plain


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n", [(32, 16, 8, 4), (16, 8, 8, 16), (16, 16, 16, 16), (32, 8, 16, 8)])
def test_staged_overrelax_bitwise(su2, n, prec):
    print(f"staged overrelaxation {n} {prec}", flush=True)
    staged, plain = _pair(su2, n, prec, 11)
    for mu in range(4):
        for par in range(2):
            su2.su2_overrelax_halfsweep(staged, mu, par)
            su2.su2_overrelax_halfsweep(plain, mu, par)
            torch.cuda.synchronize()
            assert torch.equal(staged.links, plain.links), (mu, par)
    su2.su2_overrelax(staged, 2)
    su2.su2_overrelax(plain, 2)
    # a last sweep that takes the plaquette (its classes 1-3 odd run the
    # global-memory kernel)
    m_s = su2.su2_overrelax_measured(staged, 1)
    m_p = su2.su2_overrelax_measured(plain, 1)
    torch.cuda.synchronize()
    assert torch.equal(staged.links, plain.links)
    assert torch.equal(m_s, m_p)
    f = su2.su2_get_flags(staged)
    torch.cuda.synchronize()
    assert int(f.item()) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_staged_overrelax_bitwise_64(su2, prec):
    n = (64, 64, 64, 64)
    print(f"staged overrelaxation {n} {prec}", flush=True)
    staged, plain = _pair(su2, n, prec, 1234)
    su2.su2_overrelax(staged, 1)
    su2.su2_overrelax(plain, 1)
    torch.cuda.synchronize()
    assert torch.equal(staged.links, plain.links)


def test_staged_overrelax_matches_oracle(su2):
    # and against the oracle directly, FP64, one sweep
    n = (16, 8, 8, 16)
    U0 = oracle.init_hot(n, 5)
    oracle.heatbath_sweep(n, U0, 2.3, 5, 0)
    lat = su2.Lattice(n, "f64", device="cuda", tile=-2)
    su2.from_canonical(lat, U0)
    oracle.overrelax_sweep(n, U0)
    su2.su2_overrelax(lat, 1)
    torch.cuda.synchronize()
    import numpy as np
    assert float(np.max(np.abs(su2.to_canonical(lat).numpy() - U0))) <= 1e-13


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n", [(32, 16, 8, 4), (16, 8, 8, 16), (16, 16, 16, 16), (32, 8, 16, 8)])
def test_staged_heatbath_bitwise(su2, n, prec):
    print(f"staged heat bath {n} {prec}", flush=True)
    seed = 21
    staged, plain = _pair(su2, n, prec, seed, tile=-3)
    # beta 0.5 runs the Creutz branch with many rejected lanes to compact
    for s, beta in enumerate((2.3, 0.5)):
        for mu in range(4):
            for par in range(2):
                su2.su2_heatbath_halfsweep(staged, beta, seed, 10 + s, mu, par)
                su2.su2_heatbath_halfsweep(plain, beta, seed, 10 + s, mu, par)
                torch.cuda.synchronize()
                assert torch.equal(staged.links, plain.links), (beta, mu, par)
    for s in range(2):
        su2.su2_heatbath_sweep(staged, 2.5, seed, 20 + s)
        su2.su2_heatbath_sweep(plain, 2.5, seed, 20 + s)
    su2.su2_overrelax(staged, 1)
    su2.su2_overrelax(plain, 1)
    # a heat-bath sweep that takes the plaquette (its classes 1-3 odd run the
    # global-memory kernel)
    m_s = su2.su2_heatbath_sweep_measured(staged, 2.5, seed, 30)
    m_p = su2.su2_heatbath_sweep_measured(plain, 2.5, seed, 30)
    torch.cuda.synchronize()
    assert torch.equal(staged.links, plain.links)
    assert torch.equal(m_s, m_p)
    f = su2.su2_get_flags(staged)
    torch.cuda.synchronize()
    assert int(f.item()) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_staged_heatbath_bitwise_64(su2, prec):
    # FP64 at 64^4 has no slab plan beside the heat bath's LDS: its classes
    # run the global-memory kernel, which this also checks
    n = (64, 64, 64, 64)
    print(f"staged heat bath {n} {prec}", flush=True)
    staged, plain = _pair(su2, n, prec, 1234, tile=-3)
    su2.su2_heatbath_sweep(staged, 2.3, 1234, 1)
    su2.su2_heatbath_sweep(plain, 2.3, 1234, 1)
    torch.cuda.synchronize()
    assert torch.equal(staged.links, plain.links)


def test_staged_heatbath_matches_oracle(su2):
    import numpy as np
    n = (16, 8, 8, 16)
    U0 = oracle.init_hot(n, 6)
    lat = su2.Lattice(n, "f64", device="cuda", tile=-3)
    su2.from_canonical(lat, U0)
    assert oracle.heatbath_sweep(n, U0, 2.3, 6, 0) == 0
    su2.su2_heatbath_sweep(lat, 2.3, 6, 0)
    torch.cuda.synchronize()
    assert float(np.max(np.abs(su2.to_canonical(lat).numpy() - U0))) <= 1e-12


def test_staged_overrelax_bitwise_96(su2):
    # the largest single lattice (5.4 GB of links, byte offsets beyond 4 GiB
    # in the plane loads): a staged overrelaxation sweep equals the global
    # kernel's bitwise
    n = (96, 96, 96, 96)
    print(f"staged overrelaxation {n} f32", flush=True)
    staged = su2.Lattice(n, "f32", device="cuda", tile=-2)
    plain = su2.Lattice(n, "f32", device="cuda", tile=96, tile_y=8)
    su2.su2_init_cold(plain)
    su2.su2_heatbath_sweep(plain, 2.5, 1234, 0)
    staged.links.copy_(plain.links)
    su2.su2_overrelax(staged, 1)
    su2.su2_overrelax(plain, 1)
    torch.cuda.synchronize()
    assert torch.equal(staged.links, plain.links)
