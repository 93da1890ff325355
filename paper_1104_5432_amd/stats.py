"""Monte Carlo error analysis: the Gamma method of U. Wolff, "Monte Carlo
errors with less errors", Comput. Phys. Commun. 156 (2004) 143 -- the
autocorrelation function by FFT, the automatic summation window with
S = 1.5, and the bias correction of the integrated autocorrelation time."""
import numpy as np


def autocorrelation(a):
    """Gamma(t) for t = 0..N-1 (mean removed, normalised by N - t)."""
    a = np.asarray(a, dtype=np.float64)
    N = a.size
    d = a - a.mean()
    f = np.fft.rfft(d, n=2 * N)
    acf = np.fft.irfft(f * np.conj(f), n=2 * N)[:N]
    return acf / (N - np.arange(N))


def gamma_method(a, S=1.5):
    """Return (mean, error, tau_int, window) of the series a."""
    a = np.asarray(a, dtype=np.float64)
    N = a.size
    mean = a.mean()
    gam = autocorrelation(a)
    gamma0 = gam[0]
    if not gamma0 > 0.0:
        return mean, 0.0, 0.5, 0
    tmax = N // 2
    csum = np.cumsum(gam[1:tmax + 1]) / gamma0
    window = tmax
    for W in range(1, tmax + 1):
        tau_w = 0.5 + csum[W - 1]
        if tau_w <= 0.5:
            window = W
            break
        tau = S / np.log((2 * tau_w + 1) / (2 * tau_w - 1))
        if np.exp(-W / tau) - tau / np.sqrt(W * N) < 0:
            window = W
            break
    c_total = gamma0 + 2 * gam[1:window + 1].sum()
    c_total *= 1.0 + (2 * window + 1) / N
    tau_int = max(c_total / (2 * gamma0), 0.5)
    err = np.sqrt(max(c_total, 0.0) / N)
    return mean, err, tau_int, window
