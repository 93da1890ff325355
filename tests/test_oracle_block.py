"""Pins of the oracle's learned block move (exactness of the Metropolis-
Hastings step on the marginal of a block centre).

- Bessel functions against scipy.special.ive (a separate implementation).
- The block piece identity |V_o(T)|^2 = |S_o|^2 + 1 + 2 (1/2)Tr(T S_o)
  against the oracle's staple function with T written into the lattice.
- The proposal's coefficients: c_o is the slope of the o-th factor of the
  log marginal at (1/2)Tr(T S_o) = 0 (central difference of scipy's
  Bessel function), times exp(y_o); the directions add.
- The action decomposition behind the marginal: changing a block centre and
  its six neighbours changes the brute-force Wilson action by exactly
  -beta sum_o d[(1/2)Tr(T_o V_o(T_e))].
- Colour classes: two centres of one parity and colour are >= 4 apart.
- Stationary law: repeated moves of one class (nothing else moving) make
  each centre's link follow the marginal prod_o Z(beta|V_o(T)|); checked
  against a direct quadrature over SU(2).
- The redraw of the integrated links: after a class of moves every
  neighbour link follows its heat-bath conditional law given the rest
  (probability-integral transform against the exact CDF).
"""
import itertools

import numpy as np
import pytest
from scipy import special, stats

import oracle
from tests import stats_util


def _site(n, x, y, z, t):
    return x + n[0] * (y + n[1] * (z + n[2] * t))


def test_bessel_against_scipy():
    xs = np.concatenate([np.logspace(-10, 0, 25), np.linspace(0.5, 200, 200)])
    for k in (1, 2):
        for x in xs:
            assert abs(oracle.bessel_ive(k, x) - special.ive(k, x)) <= 1e-14 * special.ive(k, x)
    for a in (1e-3, 0.7, 2.3, 9.0, 40.0):
        assert abs(oracle.log_z(a) - np.log(2 * special.iv(1, a) / a)) <= 1e-13 * max(1, abs(oracle.log_z(a)))
        assert abs(oracle.bessel_ratio(a) - special.iv(2, a) / special.iv(1, a)) <= 1e-14
    assert oracle.log_z(0.0) == 0.0 and oracle.bessel_ratio(0.0) == 0.0


def test_block_piece_identity():
    n = (8, 8, 8, 2)
    U = oracle.init_hot(n, 5)
    rng = np.random.default_rng(3)
    for _ in range(10):
        x, y, z, t = [int(v) for v in rng.integers(0, 8, 3)] + [int(rng.integers(0, 2))]
        e = _site(n, x, y, z, t)
        T = rng.normal(size=4)
        T /= np.linalg.norm(T)
        U[t, z, y, x, 3] = T
        for d in range(6):
            S = oracle.block_piece(n, U, e, d)
            i, s = d // 2, (+1 if d % 2 else -1)
            o = oracle.neighbor(n, e, i, s)
            V = oracle.staple(n, U, o, 3)
            lhs = float(V @ V)
            rhs = float(S @ S) + 1 + 2 * oracle.qmul(T, S)[0]
            assert abs(lhs - rhs) <= 1e-12, (d, lhs, rhs)


def test_block_proposal_is_the_slope_of_the_marginal():
    # The proposal's effective staple M = sum_o c_o S_o takes for c_o (at
    # y_o = 0) the slope of the o-th factor of the marginal,
    # log Z(beta sqrt(|S_o|^2 + 1 + 2w)) in w = (1/2)Tr(T S_o), at w = 0,
    # times exp(y_o).  Each direction is isolated by giving the others
    # y = -60 (weight e^-60); the slope comes from a central difference of
    # scipy's Bessel function, not from the oracle's.
    n, beta = (8, 8, 8, 2), 2.3
    U = oracle.init_hot(n, 21)
    rng = np.random.default_rng(8)
    h = 1e-5
    for _ in range(6):
        x, y, z, t = [int(v) for v in rng.integers(0, 8, 3)] + [int(rng.integers(0, 2))]
        e = _site(n, x, y, z, t)
        S = [oracle.block_piece(n, U, e, d) for d in range(6)]
        for d in range(6):
            s2 = float(S[d] @ S[d])

            def f(w):
                a = beta * np.sqrt(s2 + 1 + 2 * w)
                return np.log(2 * special.ive(1, a) / a) + a

            slope = (f(h) - f(-h)) / (2 * h)
            for yd in (0.0, 0.7, -1.3):
                y6 = np.full(6, -60.0)
                y6[d] = yd
                M = oracle.block_proposal(n, U, e, beta, y6)
                want = slope * np.exp(yd) * S[d]
                assert np.allclose(M, want, rtol=1e-7, atol=1e-7 * np.linalg.norm(want)), (d, yd, M, want)
        # all directions at once: the sum of the isolated ones
        y6 = rng.normal(scale=0.5, size=6)
        M = oracle.block_proposal(n, U, e, beta, y6)
        parts = [oracle.block_proposal(n, U, e, beta, np.where(np.arange(6) == d, y6, -60.0)) for d in range(6)]
        assert np.allclose(M, np.sum(parts, 0), rtol=1e-12, atol=1e-12)


def test_block_action_decomposition():
    n = (8, 8, 8, 2)
    beta = 2.3
    U = oracle.init_hot(n, 6)
    rng = np.random.default_rng(4)
    flat = U.reshape(-1, 4, 4)
    vol = int(np.prod(n))
    for _ in range(5):
        x, y, z, t = [int(v) for v in rng.integers(0, 8, 3)] + [int(rng.integers(0, 2))]
        e = _site(n, x, y, z, t)
        block = [e] + [oracle.neighbor(n, e, d // 2, +1 if d % 2 else -1) for d in range(6)]

        def local(Ucfg):
            # sum over the six neighbours of (1/2)Tr(T_o V_o) (contains every plaquette of the block once)
            return sum(oracle.qmul(Ucfg.reshape(-1, 4, 4)[o, 3], oracle.staple(n, Ucfg, o, 3))[0]
                       for o in block[1:])

        S0 = beta * 6 * vol * (1 - oracle.plaquette(n, U)[0])
        l0 = local(U)
        for b in block:
            q = rng.normal(size=4)
            flat[b, 3] = q / np.linalg.norm(q)
        S1 = beta * 6 * vol * (1 - oracle.plaquette(n, U)[0])
        assert abs((S1 - S0) + beta * (local(U) - l0)) <= 1e-9 * max(1.0, S0)


def test_colour_classes_do_not_interact():
    for n in ((8, 8, 8, 2), (16, 16, 16, 4)):
        cells = {}
        for x, y, z in itertools.product(range(n[0]), range(n[1]), range(n[2])):
            cells.setdefault(((x + y + z) % 2, oracle.block_colour(x, y, z)), []).append((x, y, z))
        assert len(cells) == 16
        for pts in cells.values():
            P = np.array(pts)
            d = np.abs(P[:, None, :] - P[None, :, :])
            d = np.minimum(d, np.array(n[:3]) - d).sum(-1)
            np.fill_diagonal(d, 99)
            assert d.min() >= 4


def _haar_grid(nchi=40, ntheta=20, nphi=40):
    # T = (cos c, sin c (sin th cos ph, sin th sin ph, cos th)), Haar ~ sin^2 c sin th
    xc, wc = np.polynomial.legendre.leggauss(nchi)
    chi = 0.5 * np.pi * (xc + 1)
    wchi = 0.5 * np.pi * wc * np.sin(chi) ** 2
    xt, wt = np.polynomial.legendre.leggauss(ntheta)     # in cos(theta)
    ph = 2 * np.pi * (np.arange(nphi) + 0.5) / nphi
    C, CT, PH = np.meshgrid(chi, xt, ph, indexing="ij")
    W = np.meshgrid(wchi, wt, np.full(nphi, 2 * np.pi / nphi), indexing="ij")
    w = (W[0] * W[1] * W[2]).ravel()
    st = np.sqrt(1 - CT ** 2)
    T = np.stack([np.cos(C), np.sin(C) * st * np.cos(PH), np.sin(C) * st * np.sin(PH), np.sin(C) * CT], -1)
    return T.reshape(-1, 4), w / w.sum()


@pytest.mark.slow
def test_block_move_samples_the_marginal():
    n, beta, seed = (8, 8, 8, 2), 2.3, 91
    U = oracle.init_hot(n, seed)
    for s in range(20):
        oracle.heatbath_sweep(n, U, beta, seed, s)
    rng = np.random.default_rng(8)
    y = rng.normal(scale=0.3, size=(2, 8, 8, 8, 6))        # an arbitrary (untrained) network output
    # four centres of class (parity 0, colour 0) and their exact marginal
    cen = [(x, yy, z, t) for t in range(2) for z in range(8) for yy in range(8) for x in range(8)
           if (x + yy + z) % 2 == 0 and oracle.block_colour(x, yy, z) == 0][:4]
    grid, w = _haar_grid()
    ref, probes = [], []
    for (x, yy, z, t) in cen:
        e = _site(n, x, yy, z, t)
        S = np.array([oracle.block_piece(n, U, e, d) for d in range(6)])
        s2 = (S * S).sum(1)
        # (1/2)Tr(T S) = t0 s0 - t.s
        hts = grid[:, :1] * S[None, :, 0] - (grid[:, None, 1:] * S[None, :, 1:]).sum(-1)
        a = beta * np.sqrt(np.maximum(s2[None, :] + 1 + 2 * hts, 0))
        logp = np.log(special.ive(1, a) * 2 / np.maximum(a, 1e-300)) + a
        logp = logp.sum(1)
        p = w * np.exp(logp - logp.max())
        p /= p.sum()
        probe = S.sum(0) / np.linalg.norm(S.sum(0))             # a test direction
        f = grid[:, 0] * probe[0] - grid[:, 1:] @ probe[1:]
        ref.append(float((p * f).sum()))
        probes.append((e, probe, t, z, yy, x))
    series = [[] for _ in cen]
    acc = 0
    for step in range(3000):
        f, a_ = oracle.block_move(n, U, beta, seed, step, 0, 0, y)
        acc += a_
        for j, (e, probe, t, z, yy, x) in enumerate(probes):
            T = U[t, z, yy, x, 3]
            series[j].append(T[0] * probe[0] - T[1:] @ probe[1:])
    rate = acc / (3000 * 128)
    assert 0.05 < rate < 1.0, rate
    for j in range(len(cen)):
        m, err, tau, _ = stats_util.gamma_error(np.array(series[j]))
        assert abs(m - ref[j]) <= 4 * err + 1e-3, (j, m, ref[j], err, tau)


def test_block_move_redraws_the_neighbours_from_their_conditional_law():
    # After a class of block moves each neighbour temporal link T(o) was drawn
    # by heat bath given everything else, the centre after its decision
    # included, and nothing in its staple moves later in the class (another
    # centre of the class is >= 3 away from o, its neighbours >= 2, and the
    # staple of a temporal link holds temporal links of its own slice at
    # distance 1 only).  So F_alpha(w0) ~ U(0,1) with w0 = (1/2)Tr(T(o) Vhat_o),
    # alpha = beta |V_o|.  A redraw at the wrong coupling, or none, fails.
    n, beta, seed = (8, 8, 8, 4), 2.3, 17
    U = oracle.init_hot(n, seed)
    for s in range(10):
        assert oracle.heatbath_sweep(n, U, beta, seed, s) == 0
    rng = np.random.default_rng(3)
    y = rng.normal(scale=0.3, size=(n[3], n[2], n[1], n[0], 6))
    pit = []
    for step in range(3):
        for p, k in ((0, 0), (1, 3), (0, 5), (1, 6)):
            f, _ = oracle.block_move(n, U, beta, seed, step, p, k, y)
            assert f == 0
            flat = U.reshape(-1, 4, 4)
            for t, z, yy, x in itertools.product(range(n[3]), range(n[2]), range(n[1]), range(n[0])):
                if (x + yy + z) % 2 != p or oracle.block_colour(x, yy, z) != k:
                    continue
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    o = _site(n, (x + dx) % n[0], (yy + dy) % n[1], (z + dz) % n[2], t)
                    V = oracle.staple(n, U, o, 3)
                    kv = np.linalg.norm(V)
                    w0 = oracle.qmul(flat[o, 3], V / kv)[0]
                    pit.append(float(stats_util.x0_cdf(np.array(beta * kv), np.array(w0))))
    pit = np.array(pit)
    assert pit.size >= 3000
    assert stats.kstest(pit, "uniform").pvalue > 1e-4
