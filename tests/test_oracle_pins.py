"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each test states what fixes the expected value: a separately written library
routine, a closed form, an invariant of the method, an exact conditional law,
or a known limit.  Statistical tests use fixed seeds chosen in advance.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import special, stats

import oracle
from tests import stats_util

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")     # build output of the test's helper program


# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11) against PyTorch's host Philox engine
# --------------------------------------------------------------------------
def _torch_philox_ref():
    import torch.utils.cpp_extension as ce
    exe = os.path.join(BUILD, "ref_torch_philox")
    src = os.path.join(HERE, "ref_torch_philox.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        os.makedirs(BUILD, exist_ok=True)
        subprocess.run(["g++", "-std=c++17", "-O1", "-I" + ce.include_paths()[0], "-o", exe, src],
                       check=True)
    return exe


def test_philox_matches_independent_engine():
    rng = np.random.default_rng(20110220)
    cases = [[0] * 6, [0xffffffff] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 0, 1]]
    cases += rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64).tolist()
    # counters as the method uses them: (site, mu + 4 kind, sweep, 4 attempt + draw)
    for site in (0, 1, 4095, 123457):
        for c1 in (0, 3, 4, 7, 12, 16 + 5):
            for c3 in (0, 1, 2, 4, 5, 4 * 4095 + 1):
                cases.append([site, c1, 17, c3, 1234, 0])
    text = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
    out = subprocess.run([_torch_philox_ref()], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = oracle.philox4x32_10(c[:4], c[4:])
        assert got == ref, (c, got, ref)


def test_philox_uniformity():
    # 2^15 calls -> 2^17 words; mean/variance of u01 and KS against U(0,1).
    u = []
    for i in range(1 << 15):
        r = oracle.philox4x32_10([i, 5, 9, 0], [1234, 0])
        u.append(oracle.u01_f64(r[0], r[1]))
        u.append(oracle.u01_f64(r[2], r[3]))
    u = np.array(u)
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    assert stats.kstest(u, "uniform").pvalue > 1e-4


# --------------------------------------------------------------------------
# uniform conversions: closed-form edges
# --------------------------------------------------------------------------
def test_u01_edges():
    assert oracle.u01_f64(0, 0) == 2.0 ** -53
    assert oracle.u01_f64(0xffffffff, 0xffffffff) == 1.0 - 2.0 ** -53
    # the low 12 bits of the odd word are dropped
    assert oracle.u01_f64(0, 0xfff) == 2.0 ** -53
    assert oracle.u01_f64(0, 0x1000) == 3 * 2.0 ** -53
    assert oracle.u01_f64(0x80000000, 0) == 0.5 + 2.0 ** -53
    assert np.float32(oracle.u01_f32(0)) == np.float32(2.0 ** -24)
    assert np.float32(oracle.u01_f32(0xffffffff)) == np.float32(1.0 - 2.0 ** -24)
    assert np.float32(oracle.u01_f32(0x1ff)) == np.float32(2.0 ** -24)
    # the FP32 uniform is the FP64 uniform of the same word pair to 23 bits
    for w in (0x12345678, 0x9abcdef0, 0xdeadbeef):
        assert abs(oracle.u01_f32(w) - oracle.u01_f64(w, 0x55555555)) < 2.0 ** -23


# --------------------------------------------------------------------------
# quaternion algebra against 2x2 complex matrices
# --------------------------------------------------------------------------
def _mat(q):
    a0, a1, a2, a3 = q
    return np.array([[a0 + 1j * a3, a2 + 1j * a1], [-a2 + 1j * a1, a0 - 1j * a3]])


def test_quaternion_algebra_matches_matrices():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = rng.normal(size=4), rng.normal(size=4)
        assert np.allclose(_mat(oracle.qmul(a, b)), _mat(a) @ _mat(b), atol=1e-14, rtol=0)
        assert np.allclose(_mat(oracle.qdag(a)), _mat(a).conj().T, atol=0, rtol=0)
        assert abs(0.5 * np.trace(_mat(a)).real - a[0]) < 1e-15
        # unit quaternions are SU(2): unitary with determinant one
        q = a / np.linalg.norm(a)
        M = _mat(q)
        assert np.allclose(M @ M.conj().T, np.eye(2), atol=1e-15)
        assert abs(np.linalg.det(M) - 1) < 1e-15


# --------------------------------------------------------------------------
# geometry: checkerboard independence, by perturbation of a black box
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [(4, 4, 4, 4), (4, 4, 4, 2), (2, 4, 6, 4)])
def test_checkerboard_classes_are_independent(n):
    U = oracle.init_hot(n, 77)
    vol = int(np.prod(n))
    flat = U.reshape(vol, 4, 4)
    for mu in range(4):
        for p in range(2):
            cls = [i for i in range(vol) if oracle.parity(n, i) == p]
            base = np.array([oracle.staple(n, U, i, mu) for i in cls])
            j = cls[len(cls) // 3]
            saved = flat[j, mu].copy()
            flat[j, mu] = [0.3, -0.2, 0.9, 0.1]
            new = np.array([oracle.staple(n, U, i, mu) for i in cls])
            flat[j, mu] = saved
            assert np.array_equal(new, base), (mu, p)
            # the staples do depend on the other links: perturbing a link of
            # the opposite parity changes some staple of this class
            k = next(i for i in range(vol) if oracle.parity(n, i) != p)
            saved_k = flat[k, mu].copy()
            flat[k, mu] = [0.3, -0.2, 0.9, 0.1]
            new2 = np.array([oracle.staple(n, U, i, mu) for i in cls])
            flat[k, mu] = saved_k
            assert not np.array_equal(new2, base)


# --------------------------------------------------------------------------
# staple orientation: brute-force change of the total Wilson action
# --------------------------------------------------------------------------
def _total_action(n, U, beta):
    p, _ = oracle.plaquette(n, U)
    return beta * 6 * int(np.prod(n)) * (1.0 - p)


@pytest.mark.parametrize("n", [(4, 6, 4, 8), (4, 4, 4, 4)])
def test_staple_gives_local_action_change(n):
    beta = 2.3
    rng = np.random.default_rng(5)
    U = oracle.init_hot(n, 99)
    vol = int(np.prod(n))
    flat = U.reshape(vol, 4, 4)
    S0 = _total_action(n, U, beta)
    for _ in range(12):
        i, mu = int(rng.integers(vol)), int(rng.integers(4))
        V = oracle.staple(n, U, i, mu)
        old = flat[i, mu].copy()
        new = rng.normal(size=4)
        new /= np.linalg.norm(new)
        flat[i, mu] = new
        S1 = _total_action(n, U, beta)
        # local action -(beta/2) Tr(U V) = -beta * scalar part of U V
        pred = -beta * (oracle.qmul(new, V)[0] - oracle.qmul(old, V)[0])
        assert abs((S1 - S0) - pred) < 1e-10 * max(1.0, abs(S0)), (i, mu)
        S0 = S1


# --------------------------------------------------------------------------
# observables: closed forms
# --------------------------------------------------------------------------
def test_cold_start_observables():
    n = (4, 6, 4, 8)
    U = oracle.init_cold(n)
    p, planes = oracle.plaquette(n, U)
    assert p == 1.0 and np.all(planes == 1.0)
    assert oracle.polyakov(n, U) == (1.0, 1.0)
    assert np.all(oracle.polyakov_corr(n, U) == 1.0)


def test_plaquette_constant_field_closed_form():
    # U_x(x,y,z,t) = exp(i theta y sigma3), all other links 1: the (x,y)
    # plaquettes equal exp(-i theta sigma3) (half trace cos theta), all other
    # planes are 1.  theta = 2 pi m / Ny keeps the field periodic.
    n = (4, 6, 4, 2)
    nx, ny, nz, nt = n
    theta = 2 * np.pi * 2 / ny
    U = oracle.init_cold(n)
    for y in range(ny):
        U[:, :, y, :, 0] = [np.cos(theta * y), 0, 0, np.sin(theta * y)]
    p, planes = oracle.plaquette(n, U)
    assert np.allclose(planes, [np.cos(theta), 1, 1, 1, 1, 1], atol=1e-15)
    assert abs(p - (np.cos(theta) + 5) / 6) < 1e-15


def test_polyakov_closed_forms():
    n = (8, 6, 4, 5)
    nx, ny, nz, nt = n
    # all temporal links at a spatial site equal (cos th, sin th n): L = cos(Nt th)
    U = oracle.init_cold(n)
    th = 0.37
    nvec = np.array([0.48, 0.6, 0.64])
    U[:, :, :, :, 3] = np.concatenate([[np.cos(th)], np.sin(th) * nvec])
    L = oracle.polyakov_field(n, U)
    assert np.allclose(L, np.cos(nt * th), atol=1e-14)
    # L(x) = cos(2 pi x / Nx) via one temporal link per site:
    # C(r) = (1/3) (cos(2 pi r / Nx) / 2 + 1)
    U = oracle.init_cold(n)
    for x in range(nx):
        a = 2 * np.pi * x / nx
        U[2, :, :, x, 3] = [np.cos(a), 0, np.sin(a), 0]
    C = oracle.polyakov_corr(n, U)
    r = np.arange(1, min(n[:3]) // 2 + 1)
    assert np.allclose(C, (np.cos(2 * np.pi * r / nx) / 2 + 1) / 3, atol=1e-14)
    m, ma = oracle.polyakov(n, U)
    assert abs(m) < 1e-15 and abs(ma - np.mean(np.abs(np.cos(2 * np.pi * np.arange(nx) / nx)))) < 1e-15
    # the same along y and along z (distinct extents, so a shift taken modulo
    # the wrong extent shows): C(r) = (1/3) (1 + cos(2 pi r / N_axis) / 2)
    for axis, na in ((1, ny), (2, nz)):
        U = oracle.init_cold(n)
        for c in range(na):
            a = 2 * np.pi * c / na
            idx = (2, c, slice(None), slice(None), 3) if axis == 2 else (2, slice(None), c, slice(None), 3)
            U[idx] = [np.cos(a), np.sin(a), 0, 0]
        C = oracle.polyakov_corr(n, U)
        assert np.allclose(C, (1 + np.cos(2 * np.pi * r / na) / 2) / 3, atol=1e-14), axis
    # centre transformation on odd spatial sites: C(r) -> (-1)^r on a cold start
    U = oracle.init_cold(n)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if (x + y + z) % 2:
                    U[0, z, y, x, 3] = [-1, 0, 0, 0]
    C = oracle.polyakov_corr(n, U)
    assert np.allclose(C, (-1.0) ** r, atol=0)
    # that flip is not a symmetry of the action: the three (i,t) plaquettes at
    # t = 0 become -1 at every spatial site, so <P> = 1 - 1/Nt
    assert abs(oracle.plaquette(n, U)[0] - (1 - 1 / nt)) < 1e-15


# --------------------------------------------------------------------------
# hot start: Haar measure on the 3-sphere
# --------------------------------------------------------------------------
def test_hot_start_is_haar():
    n = (16, 16, 16, 16)
    U = oracle.init_hot(n, 1234)
    q = U.reshape(-1, 4)
    N = q.shape[0]
    assert np.max(np.abs((q * q).sum(1) - 1.0)) < 1e-15
    assert np.all(np.abs(q.mean(0)) < 5 * np.sqrt(0.25 / N))
    assert np.all(np.abs((q * q).mean(0) - 0.25) < 5 * np.sqrt((1 / 8 - 1 / 16) / N))
    assert abs((q[:, 0] ** 4).mean() - 1 / 8) < 5 * np.sqrt((5 / 128 - 1 / 64) / N)
    for k in range(4):
        assert stats.kstest(q[:, k], stats_util.haar_a0_cdf).pvalue > 1e-4
    p, _ = oracle.plaquette(n, U)
    assert abs(p) < 5 * 0.5 / np.sqrt(6 * np.prod(n))
    # lattice_id shifts the stream: different lattices, same seed, differ
    U1 = oracle.init_hot((4, 4, 4, 4), 1234, lattice_id=1)
    U0 = oracle.init_hot((4, 4, 4, 4), 1234, lattice_id=0)
    assert not np.allclose(U0, U1)


# --------------------------------------------------------------------------
# heat bath: the conditional law of one link
# --------------------------------------------------------------------------
def test_x0_cdf_helper_against_bessel():
    # the quadrature CDF used below: normalisation pi I1(a)/a, mean I2/I1
    for a in (0.6, 1.8, 3.0, 13.8, 36.0):
        norm = stats_util.x0_norm_scaled(np.array(a))
        assert abs(norm - np.pi * special.ive(1, a) / a) < 1e-12 * norm
        t = np.linspace(-1, 1, 200001)
        cdf = stats_util.x0_cdf(np.full_like(t, a), t)
        mean = 1.0 - np.trapezoid(cdf, t)   # E[t] = 1 - integral of F over [-1, 1]
        assert abs(mean - special.ive(2, a) / special.ive(1, a)) < 1e-6


@pytest.mark.parametrize("beta", [0.1, 0.3, 0.5, 2.3, 6.0])
def test_single_link_sampler_law(beta):
    # Cold start: every staple is 6 * identity, so k = 6, Vhat = 1 and the
    # first half-sweep writes U = X with a0 = x0 drawn at alpha = 6 beta:
    # alpha = 0.6, 1.8 use the Creutz branch, 3, 13.8, 36 Kennedy-Pendleton.
    n = (16, 16, 16, 8)
    U = oracle.init_cold(n)
    flags = oracle.heatbath_halfsweep(n, U, beta, 4321, 0, 0, 0)
    assert flags == 0
    flat = U.reshape(-1, 4, 4)
    par = np.add.reduce(np.indices((n[3], n[2], n[1], n[0])), axis=0).reshape(-1) % 2
    upd = flat[par == 0, 0]
    # nothing else moved
    assert np.all(flat[par == 1, 0] == [1, 0, 0, 0])
    assert np.all(flat[:, 1:] == [1, 0, 0, 0])
    alpha = 6 * beta
    x0 = upd[:, 0]
    N = x0.size
    assert stats.kstest(x0, lambda w: stats_util.x0_cdf(np.full_like(w, alpha), w)).pvalue > 1e-4
    mean = special.ive(2, alpha) / special.ive(1, alpha)
    assert abs(x0.mean() - mean) < 5 * x0.std() / np.sqrt(N)
    # unit length and isotropic direction
    assert np.max(np.abs((upd * upd).sum(1) - 1)) < 1e-15
    v = upd[:, 1:] / np.linalg.norm(upd[:, 1:], axis=1, keepdims=True)
    assert np.all(np.abs(v.mean(0)) < 5 * np.sqrt(1 / 3 / N))
    assert np.all(np.abs((v * v).mean(0) - 1 / 3) < 5 * np.sqrt(4 / 45 / N))
    # cos(theta) = v_3 is uniform on [-1, 1]
    assert stats.kstest(v[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-4


def test_heatbath_at_zero_beta_draws_haar_links():
    # beta = 0: the local weight is flat, so an updated link is Haar
    # distributed whatever its staple and its old value (the Creutz branch
    # with alpha < 1e-8 draws x0 uniform and accepts with sqrt(1 - x0^2))
    n = (16, 16, 16, 8)
    U = oracle.init_hot(n, 77)
    oracle.heatbath_sweep(n, U, 2.3, 77, 0)          # a non-trivial configuration
    old = U.copy()
    flags = oracle.heatbath_halfsweep(n, U, 0.0, 77, 1, 1, 1)
    assert flags == 0
    flat, prev = U.reshape(-1, 4, 4), old.reshape(-1, 4, 4)
    par = np.add.reduce(np.indices((n[3], n[2], n[1], n[0])), axis=0).reshape(-1) % 2
    q = flat[par == 1, 1]
    N = q.shape[0]
    assert np.max(np.abs((q * q).sum(1) - 1.0)) < 1e-15
    for k in range(4):
        assert stats.kstest(q[:, k], stats_util.haar_a0_cdf).pvalue > 1e-4
    assert np.all(np.abs(q.mean(0)) < 5 * np.sqrt(0.25 / N))
    # independent of the link it replaces: <Tr(U_new U_old^+)/2> = 0
    tr = (q * prev[par == 1, 1]).sum(1)
    assert abs(tr.mean()) < 5 * np.sqrt(0.25 / N)
    # nothing else moved
    assert np.array_equal(flat[par == 0], prev[par == 0])
    assert np.array_equal(flat[:, [0, 2, 3]], prev[:, [0, 2, 3]])


def test_heatbath_at_huge_beta_stays_exact():
    # beta = 1e6 (alpha ~ 1e6-1e7): Kennedy-Pendleton with lambda^2 ~ 1e-7;
    # 1 - x0 = 2 lambda^2 is formed without cancellation, so its mean over
    # the updated links matches 1 - I2(alpha)/I1(alpha) ~ 3/(2 alpha), and
    # every link stays finite and unit
    n = (16, 16, 16, 8)
    beta = 1e6
    U = oracle.init_cold(n)
    assert oracle.heatbath_halfsweep(n, U, beta, 5, 0, 0, 0) == 0
    flat = U.reshape(-1, 4, 4)
    par = np.add.reduce(np.indices((n[3], n[2], n[1], n[0])), axis=0).reshape(-1) % 2
    upd = flat[par == 0, 0]
    assert np.all(np.isfinite(upd)) and np.max(np.abs((upd * upd).sum(1) - 1.0)) < 1e-15
    alpha = 6 * beta                                  # cold start: k = 6
    one_minus = 1.0 - upd[:, 0]
    expect = 1.0 - special.ive(2, alpha) / special.ive(1, alpha)
    assert abs(expect - 1.5 / alpha) < 1e-3 * expect
    # the vector part: |x|^2 = 1 - x0^2 to the rounding of x0 (ulp(1) ~ 1.1e-16)
    xv = (upd[:, 1:] ** 2).sum(1)
    assert np.max(np.abs(xv - one_minus * (2.0 - one_minus))) < 4e-16
    # the law: the mean of 1 - x0, from |x|^2 / 2 = 2 lambda^2 (1 - lambda^2),
    # which is free of the rounding of x0 near 1
    N = xv.size
    assert abs(xv.mean() / 2 - expect) < 5 * (xv / 2).std() / np.sqrt(N)
    assert abs(one_minus.mean() - expect) < 5 * one_minus.std() / np.sqrt(N)


@pytest.mark.parametrize("beta", [0.3, 2.3])
def test_single_precision_heatbath_law_and_agreement(beta):
    # The oracle's single-precision half-sweep (decisions in the precisions
    # of the FP32 path) samples the same law -- KS against the exact density
    # from a cold start (Creutz at alpha = 1.8, Kennedy-Pendleton at 13.8) --
    # and, from an FP32-rounded thermalised configuration, agrees with the
    # FP64 half-sweep link by link to FP32 rounding except where a decision
    # flips between 23-bit and 52-bit uniforms.
    n = (16, 16, 16, 8)
    U = oracle.init_cold(n)
    assert oracle.heatbath_halfsweep_f32(n, U, beta, 4321, 0, 0, 0) == 0
    assert np.array_equal(U.astype(np.float32).astype(np.float64), U)
    par = np.add.reduce(np.indices((n[3], n[2], n[1], n[0])), axis=0).reshape(-1) % 2
    upd = U.reshape(-1, 4, 4)[par == 0, 0]
    assert np.max(np.abs((upd * upd).sum(1) - 1.0)) < 6e-7     # a few FP32 ulp
    x0 = upd[:, 0]
    alpha = 6 * beta
    assert stats.kstest(x0, lambda w: stats_util.x0_cdf(np.full_like(w, alpha), w)).pvalue > 1e-4
    mean = special.ive(2, alpha) / special.ive(1, alpha)
    assert abs(x0.mean() - mean) < 5 * x0.std() / np.sqrt(x0.size)

    m = (8, 8, 8, 8)
    T = oracle.init_hot(m, 3)
    for s in range(3):
        oracle.heatbath_sweep(m, T, 2.3, 3, s)
    T = T.astype(np.float32).astype(np.float64)
    a, b = T.copy(), T.copy()
    oracle.heatbath_halfsweep_f32(m, a, beta, 99, 4, 1, 0)
    oracle.heatbath_halfsweep(m, b, beta, 99, 4, 1, 0)
    d = np.max(np.abs(a - b), axis=-1)
    assert np.mean(d > 5e-5) <= 1e-3 and np.median(d[d > 0]) < 1e-6


@pytest.mark.parametrize("beta,mu,p", [(2.3, 2, 1), (0.4, 3, 0), (1.0, 1, 1)])
def test_heatbath_pit_at_equilibrium(beta, mu, p):
    # After a half-sweep of class (mu, p) the staples of that class are
    # unchanged, so each updated link must satisfy F_alpha(w0) ~ U(0,1) with
    # w0 = (1/2) Tr(U Vhat), alpha = beta |V|.  beta = 0.4 and 1.0 mix the
    # Creutz and Kennedy-Pendleton branches around alpha = 2.
    n = (8, 8, 8, 8)
    U = oracle.init_hot(n, 31)
    for s in range(8):
        assert oracle.heatbath_sweep(n, U, beta, 31, s) == 0
    assert oracle.heatbath_halfsweep(n, U, beta, 31, 8, mu, p) == 0
    vol = int(np.prod(n))
    flat = U.reshape(vol, 4, 4)
    pit = []
    alphas = []
    for i in range(vol):
        if oracle.parity(n, i) != p:
            continue
        V = oracle.staple(n, U, i, mu)
        k = np.linalg.norm(V)
        w0 = oracle.qmul(flat[i, mu], V / k)[0]
        pit.append(stats_util.x0_cdf(np.array(beta * k), np.array(w0)))
        alphas.append(beta * k)
    pit = np.array(pit, dtype=float)
    assert stats.kstest(pit, "uniform").pvalue > 1e-4
    if beta < 2:
        assert min(alphas) < 2 < max(alphas)


def test_heatbath_is_deterministic_and_resumable():
    n = (4, 4, 4, 6)
    A = oracle.init_hot(n, 1234)
    B = A.copy()
    for s in range(4):
        oracle.heatbath_sweep(n, A, 2.3, 1234, s)
    for s in range(2):
        oracle.heatbath_sweep(n, B, 2.3, 1234, s)
    C = B.copy()  # "checkpoint"
    for s in range(2, 4):
        oracle.heatbath_sweep(n, C, 2.3, 1234, s)
    assert np.array_equal(A, C)
    # a different sweep index draws different numbers
    D = B.copy()
    oracle.heatbath_sweep(n, D, 2.3, 1234, 7)
    assert not np.array_equal(D, C)


def test_nonfinite_staple_is_flagged():
    n = (4, 4, 4, 4)
    U = oracle.init_hot(n, 3)
    U[0, 0, 0, 1, 1] = [np.nan, 0, 0, 0]   # a y-link at site (1,0,0,0)
    before = U.copy()
    f = oracle.heatbath_halfsweep(n, U, 2.3, 3, 0, 0, 0)
    assert f & oracle.FLAG_NONFINITE
    # the links whose staple touches the NaN are kept
    assert np.array_equal(U[0, 0, 0, 0, 0], before[0, 0, 0, 0, 0])
    f = oracle.overrelax_halfsweep(n, U, 0, 0)
    assert f & oracle.FLAG_NONFINITE


# --------------------------------------------------------------------------
# overrelaxation: invariants
# --------------------------------------------------------------------------
def test_overrelaxation_invariants():
    n = (6, 4, 4, 8)
    beta = 2.3
    U = oracle.init_hot(n, 8)
    for s in range(5):
        oracle.heatbath_sweep(n, U, beta, 8, s)
    S0 = _total_action(n, U, beta)
    for mu in range(4):
        for p in range(2):
            before = U.copy()
            assert oracle.overrelax_halfsweep(n, U, mu, p) == 0
            S1 = _total_action(n, U, beta)
            assert abs(S1 - S0) < 1e-12 * abs(S0)
            assert not np.array_equal(before, U)
            W = U.copy()
            oracle.overrelax_halfsweep(n, W, mu, p)   # applied twice: identity
            assert np.max(np.abs(W - before)) < 1e-14
    oracle.overrelax_sweep(n, U)
    assert abs(_total_action(n, U, beta) - S0) < 1e-12 * abs(S0)


def test_unitarity_is_kept_by_long_chains():
    n = (4, 4, 4, 4)
    U = oracle.init_hot(n, 11)
    for s in range(100):
        oracle.heatbath_sweep(n, U, 2.5, 11, s)
        oracle.overrelax_sweep(n, U)
    q = U.reshape(-1, 4)
    assert np.max(np.abs((q * q).sum(1) - 1)) < 1e-14


# --------------------------------------------------------------------------
# gauge invariance of every observable
# --------------------------------------------------------------------------
def test_gauge_invariance():
    n = (6, 4, 8, 4)
    U = oracle.init_hot(n, 21)
    for s in range(3):
        oracle.heatbath_sweep(n, U, 2.3, 21, s)
    p0, pl0 = oracle.plaquette(n, U)
    L0 = oracle.polyakov_field(n, U)
    C0 = oracle.polyakov_corr(n, U)
    V0 = oracle.staple(n, U, 5, 2)
    before = U.copy()
    oracle.gauge_transform(n, U, 999)
    assert np.max(np.abs(U - before)) > 0.5
    p1, pl1 = oracle.plaquette(n, U)
    assert abs(p1 - p0) < 1e-13 and np.max(np.abs(pl1 - pl0)) < 1e-13
    assert np.max(np.abs(oracle.polyakov_field(n, U) - L0)) < 1e-13
    assert np.max(np.abs(oracle.polyakov_corr(n, U) - C0)) < 1e-13
    # the staple's local action with its own link is gauge invariant too
    assert abs(oracle.qmul(U.reshape(-1, 4, 4)[5, 2], oracle.staple(n, U, 5, 2))[0]
               - oracle.qmul(before.reshape(-1, 4, 4)[5, 2], V0)[0]) < 1e-13


# --------------------------------------------------------------------------
# strong and weak coupling limits
# --------------------------------------------------------------------------
@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.1, 0.25, 0.5])
def test_strong_coupling_plaquette(beta):
    # leading character expansion: <P> = u + O(u^5), u = I2(beta)/I1(beta)
    n = (8, 8, 8, 8)
    U = oracle.init_hot(n, 600 + int(beta * 100))
    series, planes = [], []
    for s in range(160):
        oracle.heatbath_sweep(n, U, beta, 600, s)
        if s >= 10:
            p, pl = oracle.plaquette(n, U)
            series.append(p)
            planes.append(pl)
    u = special.iv(2, beta) / special.iv(1, beta)
    mean, err, tau, _ = stats_util.gamma_error(series)
    assert abs(mean - u) < 3 * err + 6 * u ** 5, (mean, u, err)
    # hypercubic symmetry: plane averages agree within errors
    planes = np.array(planes)
    pm = planes.mean(0)
    pe = np.array([stats_util.gamma_error(planes[:, k])[1] for k in range(6)])
    assert np.all(np.abs(pm - pm.mean()) < 4 * pe + 1e-12)


@pytest.mark.slow
def test_weak_coupling_plaquette():
    # leading perturbation theory for SU(2) in 4-D: 1 - <P> = 3/(4 beta) + O(1/beta^2);
    # fit beta (1 - <P>) = a + b / beta and require a = 3/4.
    n = (8, 8, 8, 8)
    betas = np.array([10.0, 20.0, 40.0, 80.0])
    y, e = [], []
    for beta in betas:
        U = oracle.init_cold(n)
        series = []
        for s in range(90):
            oracle.heatbath_sweep(n, U, beta, 700, s)
            oracle.overrelax_sweep(n, U)
            if s >= 20:
                series.append(beta * (1.0 - oracle.plaquette(n, U)[0]))
        m, err, _, _ = stats_util.gamma_error(series)
        y.append(m)
        e.append(err)
    y, e = np.array(y), np.array(e)
    A = np.stack([np.ones_like(betas), 1 / betas], 1) / e[:, None]
    coef, *_ = np.linalg.lstsq(A, y / e, rcond=None)
    cov = np.linalg.inv(A.T @ A)
    a, sa = coef[0], np.sqrt(cov[0, 0])
    # 1/V torus zero-mode correction is ~ 3/(4 V) relative: 2e-4 here
    assert abs(a - 0.75) < 3 * sa + 0.75 * 4 / np.prod(n), (a, sa, coef)
