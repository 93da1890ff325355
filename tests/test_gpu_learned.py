"""Learned block proposal on the GPU against the oracle.

- Network outputs and gradients: the GPU (BF16 MFMA, FP32 accumulation)
  against the FP64 reference that rounds the same operands to bfloat16.  The
  remaining difference is FP32 accumulation and the rare operand whose FP32
  value on the GPU rounds to the other bfloat16 neighbour than the
  reference's (each moves one product by ~2^-9 of its size): bound 1e-3 of
  the largest entry of each tensor.
- Block sweep: per-link parity with the oracle's move in FP64 (same network
  outputs, same random numbers; 1e-12), identical acceptance count.
- Exactness: chains with learned sweeps (any network) sample the same
  ensemble as plain heat bath: plaquette and |Polyakov loop| within 3 sigma.
"""
import numpy as np
import pytest

import oracle
from oracle import network as net
from tests import stats_util

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd as m
    return m


def _sync():
    torch.cuda.synchronize()


def _config(n, beta, seed, sweeps=3):
    U = oracle.init_hot(n, seed)
    for s in range(sweeps):
        oracle.heatbath_sweep(n, U, beta, seed, s)
    return U


def _params(seed):
    rng = np.random.default_rng(seed)
    p = net.unpack(net.init_params(seed))
    p["V"] = rng.normal(scale=0.3, size=p["V"].shape)
    p["bv"] = rng.normal(scale=0.1, size=6)
    p["b2"] = rng.normal(scale=0.1, size=32)
    return net.pack(p).astype(np.float32).astype(np.float64)


def _lat(su2, n, prec, U):
    lat = su2.Lattice(n, prec, device="cuda")
    su2.from_canonical(lat, U)
    return lat


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_network_forward_matches_reference(su2, prec):
    n = (16, 8, 8, 2)
    U = _config(n, 2.3, 5)
    params = _params(21)
    lat = _lat(su2, n, prec, U)
    Uc = su2.to_canonical(lat).numpy()
    work = su2.LPWork(n)
    p = torch.tensor(params, dtype=torch.float32, device="cuda")
    y = su2.su2_lp_forward(lat, p, work)
    _sync()
    got = y.cpu().numpy().reshape(n[3], n[2], n[1], n[0], 6)
    ref = net.forward(net.features(n, Uc), params, rnd=True)["y"]
    assert _rel(got, ref) <= 1e-3, _rel(got, ref)
    # and the rounding matters: without it the difference is visibly larger
    plain = net.forward(net.features(n, Uc), params, rnd=False)["y"]
    assert _rel(got, plain) > _rel(got, ref)


def test_loss_and_gradient_match_reference(su2):
    n, beta = (8, 8, 16, 2), 2.3
    U = _config(n, beta, 7)
    params = _params(22)
    lat = _lat(su2, n, "f64", U)
    work = su2.LPWork(n)
    p = torch.tensor(params, dtype=torch.float32, device="cuda")
    grad, loss = su2.su2_lp_loss_grad(lat, beta, p, work)
    _sync()
    cache = net.forward(net.features(n, U), params, rnd=True)
    loss_ref, dy = net.loss_and_grad_y(n, U, cache["y"], beta)
    g_ref = net.unpack(net.backward(cache, dy, params, rnd=True))
    g = net.unpack(grad.cpu().numpy().astype(np.float64))
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref), (loss.item(), loss_ref)
    for name, _ in net.SHAPES:
        if name in ("W1", "b1") and np.max(np.abs(g_ref[name])) == 0:
            continue
        assert _rel(g[name], g_ref[name]) <= 1e-3, (name, _rel(g[name], g_ref[name]))


def test_adam_matches_reference(su2):
    rng = np.random.default_rng(3)
    k = 1000
    p0, g0 = rng.normal(size=k), rng.normal(size=k)
    m0, v0 = rng.normal(size=k) * 0.1, np.abs(rng.normal(size=k)) * 0.1
    t = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (p0, g0, m0, v0)]
    su2.su2_lp_adam(t[0], t[1], t[2], t[3], 7, lr=0.01)
    _sync()
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    p1, m1, v1 = net.adam(f32(p0), f32(g0), f32(m0), f32(v0), 7, lr=0.01)
    assert np.max(np.abs(t[0].cpu().numpy() - p1)) <= 1e-5
    assert np.max(np.abs(t[2].cpu().numpy() - m1)) <= 1e-6


@pytest.mark.parametrize("n", [(8, 8, 8, 2), (16, 8, 8, 4)])
def test_block_sweep_matches_oracle(su2, n):
    beta, seed = 2.3, 31
    U = _config(n, beta, 9, sweeps=4)
    rng = np.random.default_rng(4)
    y = rng.normal(scale=0.3, size=(n[3], n[2], n[1], n[0], 6)).astype(np.float32).astype(np.float64)
    lat = _lat(su2, n, "f64", U)
    yd = torch.tensor(y.ravel(), dtype=torch.float32, device="cuda")
    acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = U.copy()
    total = 0
    for step in (5, 6):
        su2.su2_lp_sweep(lat, beta, seed, step, yd, acc)
        f, a = oracle.block_sweep(n, ref, beta, seed, step, y)
        assert f == 0
        total += a
        _sync()
        err = float(np.max(np.abs(su2.to_canonical(lat).numpy() - ref)))
        assert err <= 1e-12, (step, err)
    assert int(acc.item()) == total
    assert 0.1 * 2 * np.prod(n) < total < 2 * np.prod(n)
    f = su2.su2_get_flags(lat)
    _sync()
    assert int(f.item()) == 0


@pytest.mark.parametrize("seed,parity,colour", [(12, 1, 5), (13, 0, 2), (14, 1, 7), (15, 0, 0)])
def test_single_class_move_matches_oracle_fp32(su2, seed, parity, colour):
    # FP32 links against the FP64 oracle from the same (FP32-rounded) links:
    # every moved link (a centre and its six redrawn neighbours, ~445 per
    # class) agrees to the FP32 rounding of its staples (measured <= 3.2e-7),
    # except that one centre's accept decision (and with it its block of 7
    # links) may flip between FP32 and FP64 arithmetic on a near-tie; the
    # accepted counts then differ by at most one.
    n, beta = (8, 8, 8, 2), 2.3
    U = _config(n, beta, 10)
    lat = _lat(su2, n, "f32", U)
    U32 = su2.to_canonical(lat).numpy()
    y = np.zeros((n[3], n[2], n[1], n[0], 6))
    acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    su2.su2_lp_move(lat, beta, seed, 3, parity, colour, torch.zeros(lat.volume * 6, device="cuda"), acc)
    ref = U32.copy()
    f, accepted = oracle.block_move(n, ref, beta, seed, 3, parity, colour, y)
    _sync()
    assert f == 0
    moved = np.max(np.abs(U32 - ref), axis=-1) > 0
    assert 400 < int(moved.sum()) <= 7 * 64
    d = np.max(np.abs(su2.to_canonical(lat).numpy() - ref), axis=-1)
    big = d > 1e-5
    assert int(big.sum()) <= 7, int(big.sum())
    assert float(d[~big].max()) <= 2e-6, float(d[~big].max())
    assert abs(int(acc.item()) - accepted) <= int(big.any())


@pytest.mark.slow
def test_learned_chain_is_exact(su2):
    # 16^3 x 4 at beta 2.3 (configs of the learned-proposal workload): plain
    # heat bath against heat bath + learned sweeps with an untrained,
    # randomly perturbed network; Gamma-method errors, 3 sigma.  |L| near
    # beta_c decorrelates over ~200 heat-bath sweeps, so the chains run
    # 16000 sweeps (~75 autocorrelation times) for its error to be reliable.
    from paper_1104_5432_amd import learned
    n, beta = (16, 16, 16, 4), 2.3
    params = torch.tensor(_params(40), dtype=torch.float32, device="cuda")
    res = {}
    for name, prm in (("hb", None), ("learned", params)):
        print(f"learned-chain exactness: {name} chain", flush=True)
        lat = learned.thermalised_lattice(n, beta, 77, 100)
        r = learned.run_chain(lat, beta, 77, 16000, params=prm, first_sweep=100)
        res[name] = r
    assert 0.2 < res["learned"]["acceptance"] < 1.0
    for key in ("plaquette", "polyakov"):
        a = np.array(res["hb"][key][1000:])
        b = np.array(res["learned"][key][1000:])
        if key == "polyakov":
            a, b = np.abs(a), np.abs(b)
        ma, ea, _, _ = stats_util.gamma_error(a)
        mb, eb, _, _ = stats_util.gamma_error(b)
        z = (mb - ma) / np.hypot(ea, eb)
        print(f"{key}: hb {ma:.5f}({ea:.5f}) learned {mb:.5f}({eb:.5f}) z = {z:+.2f}", flush=True)
        assert abs(z) <= 3.0


@pytest.mark.slow
def test_training_beats_the_untrained_network(su2):
    # The method without the trained network is the same block move with
    # y = 0 (mean-field coefficients).  Training on heat-bath configurations
    # must lower the held-out loss and raise the acceptance.
    from paper_1104_5432_amd import learned
    n, beta = (16, 16, 16, 4), 2.3
    lat = learned.thermalised_lattice(n, beta, 5, 300, prec="f32")
    params, losses = learned.train(lat, beta, 5, 1500, first_sweep=300, lr=2e-3)
    untrained = learned.init_params(5)
    work = su2.LPWork(n)
    held = {"trained": [], "untrained": []}
    for s in range(20):
        su2.su2_heatbath_sweep(lat, beta, 6, 5000 + s)
        for name, prm in (("trained", params), ("untrained", untrained)):
            _, loss = su2.su2_lp_loss_grad(lat, beta, prm, work)
            held[name].append(loss.item())
    assert np.mean(held["trained"]) < np.mean(held["untrained"]), held
    acc = {}
    for name, prm in (("trained", params), ("untrained", untrained)):
        c = learned.thermalised_lattice(n, beta, 8, 100, prec="f32")
        acc[name] = learned.run_chain(c, beta, 8, 60, params=prm, first_sweep=100)["acceptance"]
    print(f"acceptance {acc}", flush=True)
    assert acc["trained"] > acc["untrained"] + 0.005, acc
