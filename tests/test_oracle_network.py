"""Pins of the reference proposal network (oracle/network.py).

- Convolutions against torch.nn.functional.conv3d with circular padding
  (FP64, CPU): a separately written library routine.
- The backward pass against torch autograd through that independent forward.
- dLoss/dy against central finite differences of the loss.
- Input features against the oracle's plaquette (plane averages, single sites).
- bfloat16 rounding on exact tie cases.
"""
import numpy as np
import pytest

import oracle
from oracle import network as net

torch = pytest.importorskip("torch")


def _torch_forward(feat, params):
    """Same network written with torch conv3d (circular padding), FP64."""
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in net.unpack(params).items()}
    x = torch.tensor(feat, dtype=torch.float64)                 # (T, Z, Y, X, C)
    a = x.permute(0, 4, 1, 2, 3)                                 # (T, C, Z, Y, X)
    for layer in (1, 2, 3):
        W = p[f"W{layer}"]                                       # [tap][ci][co], tap=(dz+1)*9+(dy+1)*3+(dx+1)
        K = W.reshape(3, 3, 3, W.shape[1], W.shape[2]).permute(4, 3, 0, 1, 2)   # (co, ci, kz, ky, kx)
        a = torch.nn.functional.pad(a, (1, 1, 1, 1, 1, 1), mode="circular")
        a = torch.tanh(torch.nn.functional.conv3d(a, K) + p[f"b{layer}"][None, :, None, None, None])
    a3 = a.permute(0, 2, 3, 4, 1)
    y = a3 @ p["V"].T + p["bv"]
    return y, p


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -2.5, 0.0, 1 + 2 ** -8 + 2 ** -20])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1.0, -2.5, 0.0, 1 + 2 ** -7])
    assert np.array_equal(net.bf16(vals), want)


def test_features_are_spatial_plaquettes():
    n = (4, 6, 4, 3)
    U = oracle.init_hot(n, 2)
    for s in range(2):
        oracle.heatbath_sweep(n, U, 2.0, 2, s)
    F = net.features(n, U)
    _, planes = oracle.plaquette(n, U)
    assert abs(F[..., 0].mean() - planes[0]) < 1e-13      # xy
    assert abs(F[..., 1].mean() - planes[1]) < 1e-13      # xz
    assert abs(F[..., 2].mean() - planes[3]) < 1e-13      # yz
    assert np.allclose(F[..., 3:6], np.roll(F[..., 0:3], -1, axis=0))
    assert np.all(F[..., 6:] == 0)
    # one site by hand: (x,y,z,t) = (1,2,3,2), plane xz
    x, y, z, t = 1, 2, 3, 2
    a = oracle.qmul(U[t, z, y, x, 0], U[t, z, y, (x + 1) % 4, 2])
    b = oracle.qmul(oracle.qdag(U[t, (z + 1) % 4, y, x, 0]), oracle.qdag(U[t, z, y, x, 2]))
    assert abs(F[t, z, y, x, 1] - oracle.qmul(a, b)[0]) < 1e-14


def test_forward_matches_torch_conv3d():
    rng = np.random.default_rng(0)
    feat = rng.normal(size=(2, 4, 6, 8, net.CIN))
    params = net.init_params(1)
    params[-6:] = rng.normal(size=6)
    p = net.unpack(params)
    p["V"] = rng.normal(size=p["V"].shape)
    params = net.pack(p)
    ours = net.forward(feat, params, rnd=False)["y"]
    ref, _ = _torch_forward(feat, params)
    assert np.max(np.abs(ours - ref.detach().numpy())) < 1e-12


def test_backward_matches_autograd():
    rng = np.random.default_rng(1)
    feat = rng.normal(size=(2, 4, 6, 4, net.CIN))
    params = net.init_params(2)
    p = net.unpack(params)
    p["V"] = rng.normal(size=p["V"].shape) * 0.3
    params = net.pack(p)
    dy = rng.normal(size=(2, 4, 6, 4, net.NDIR))
    cache = net.forward(feat, params, rnd=False)
    g = net.unpack(net.backward(cache, dy, params, rnd=False))
    y, tp = _torch_forward(feat, params)
    (y * torch.tensor(dy)).sum().backward()
    for name, _ in net.SHAPES:
        ref = tp[name].grad.numpy()
        assert np.max(np.abs(g[name] - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), name


def test_loss_gradient_matches_finite_differences():
    n, beta = (4, 4, 4, 2), 2.3
    U = oracle.init_hot(n, 3)
    for s in range(3):
        oracle.heatbath_sweep(n, U, beta, 3, s)
    rng = np.random.default_rng(5)
    y = rng.normal(scale=0.3, size=(2, 4, 4, 4, 6))
    S = oracle.block_pieces_all(n, U)
    loss, dy = net.loss_and_grad_y(n, U, y, beta, S)
    assert np.isfinite(loss)
    for idx in [(0, 1, 2, 3, 0), (1, 0, 0, 0, 5), (1, 3, 2, 1, 2)]:
        h = 1e-6
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (net.loss_and_grad_y(n, U, yp, beta, S)[0] - net.loss_and_grad_y(n, U, ym, beta, S)[0]) / (2 * h)
        assert abs(fd - dy[idx]) <= 1e-7 * max(1.0, abs(dy[idx])) + 1e-10, (idx, fd, dy[idx])


def test_bf16_rounding_changes_little():
    rng = np.random.default_rng(7)
    feat = rng.uniform(-1, 1, size=(1, 4, 4, 4, net.CIN))
    params = net.init_params(3)
    a = net.forward(feat, params, rnd=False)["a3"]
    b = net.forward(feat, params, rnd=True)["a3"]
    d = np.max(np.abs(a - b))
    assert 0 < d < 2e-2


def test_adam_first_step():
    p, g = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    p1, m, v = net.adam(p, g, np.zeros(2), np.zeros(2), 1, lr=0.1)
    # first bias-corrected step moves each parameter by lr * sign(g)
    assert np.allclose(p1, p - 0.1 * np.sign(g), atol=1e-6)
