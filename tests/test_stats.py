"""Pin of the Gamma method against an AR(1) process, whose integrated
autocorrelation time tau = (1 + rho) / (2 (1 - rho)) and variance of the
mean are known in closed form."""
import numpy as np

from paper_1104_5432_amd.stats import autocorrelation, gamma_method


def test_autocorrelation_matches_direct_sum():
    rng = np.random.default_rng(0)
    a = rng.normal(size=500)
    g = autocorrelation(a)
    d = a - a.mean()
    for t in (0, 1, 7, 100):
        assert abs(g[t] - np.dot(d[:500 - t], d[t:]) / (500 - t)) < 1e-12


def test_gamma_method_on_ar1():
    rng = np.random.default_rng(2004)
    for rho in (0.0, 0.5, 0.9):
        N = 200000
        x = np.empty(N)
        e = rng.normal(size=N)
        x[0] = e[0] / np.sqrt(1 - rho * rho)
        for i in range(1, N):
            x[i] = rho * x[i - 1] + e[i]
        mean, err, tau, _ = gamma_method(x + 3.0)
        tau_exact = (1 + rho) / (2 * (1 - rho))
        var = 1.0 / (1 - rho * rho)
        assert abs(tau - tau_exact) <= 0.08 * tau_exact + 0.02, (rho, tau, tau_exact)
        assert abs(err - np.sqrt(2 * tau_exact * var / N)) <= 0.1 * err
        assert abs(mean - 3.0) <= 5 * err


def test_gamma_error_of_the_tests_on_ar1():
    # the tests' own Gamma-method estimate (tests/stats_util.py) against the
    # AR(1) closed forms, as tightly as the package's: error within 10%,
    # tau_int within 8%; a missing factor 2 in the error, a window that
    # never opens, or no bias correction would fail at rho = 0.9
    from tests import stats_util
    rng = np.random.default_rng(2004)
    for rho in (0.0, 0.5, 0.9):
        N = 1 << 18
        x = np.empty(N)
        e = rng.normal(size=N)
        x[0] = e[0] / np.sqrt(1 - rho * rho)
        for i in range(1, N):
            x[i] = rho * x[i - 1] + e[i]
        mean, err, tau, window = stats_util.gamma_error(x + 2.0)
        tau_exact = (1 + rho) / (2 * (1 - rho))
        err_exact = np.sqrt(2 * tau_exact / (1 - rho * rho) / N)
        assert window >= 1
        assert abs(err - err_exact) <= 0.1 * err_exact, (rho, err, err_exact)
        assert abs(tau - tau_exact) <= 0.08 * tau_exact + 0.02, (rho, tau, tau_exact)
        assert abs(mean - 2.0) <= 5 * err_exact
    # constant and two-point series
    assert stats_util.gamma_error(np.full(10, 3.0))[:2] == (3.0, 0.0)
    assert stats_util.gamma_error(np.array([1.0]))[1] == 0.0
