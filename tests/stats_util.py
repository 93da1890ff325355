"""Statistics used by the statistical pins and the FP32-versus-FP64 checks
(test infrastructure: nothing here comes from the package under test).

- gamma_error: the error of the mean of an autocorrelated series by the
  Gamma method (U. Wolff, Comput. Phys. Commun. 156 (2004) 143): the
  autocovariance summed up to a window W chosen automatically (the first W
  at which exp(-W/tau) - tau/sqrt(W N) turns negative, tau the exponential
  time implied by the running tau_int, S = 1.5), with the leading bias of
  the mean's estimate removed.  Written here from the paper's definitions,
  separately from the package's implementation; pinned in
  tests/test_stats.py by the closed forms of an AR(1) process.
- x0_cdf: the exact conditional distribution function of w0 = (1/2)Tr(W)
  when W has density ~ exp(alpha w0) with respect to Haar measure on SU(2),
  i.e. w0 has density ~ sqrt(1 - w0^2) exp(alpha w0) on [-1, 1].  Computed
  by Gauss-Legendre quadrature in the angle w0 = cos(theta), where the
  integrand sin^2(theta) exp(alpha (cos(theta) - 1)) is smooth.
- haar_a0_cdf: the alpha = 0 case in closed form.
"""
import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


def gamma_error(a, S=1.5):
    """Return (mean, error, tau_int, W) of the series a by the Gamma method."""
    a = np.asarray(a, dtype=np.float64)
    n = a.size
    mean = float(a.mean())
    if n < 2:
        return mean, 0.0, 0.5, 0
    d = a - mean
    c0 = float(d @ d) / n
    if not c0 > 0.0:
        return mean, 0.0, 0.5, 0
    # running sum of the normalised autocovariance, one lag at a time
    total = c0                       # C(W) = Gamma(0) + 2 sum_{t<=W} Gamma(t)
    cov = [c0]
    w_end = n // 2
    W = w_end
    for t in range(1, w_end + 1):
        g = float(d[:-t] @ d[t:]) / (n - t)
        cov.append(g)
        total += 2.0 * g
        tau_int = total / (2.0 * c0)
        if tau_int <= 0.5:           # no positive correlation left to sum
            W = t
            break
        tau = S / np.log((2.0 * tau_int + 1.0) / (2.0 * tau_int - 1.0))
        if np.exp(-t / tau) - tau / np.sqrt(t * n) < 0.0:
            W = t
            break
    # the mean subtracted from the data lowers every Gamma(t) by C(W)/n to
    # leading order: add it back, then sum again
    cw = sum(cov[:W + 1]) * 2.0 - cov[0]
    corrected = [g + cw / n for g in cov[:W + 1]]
    cw = 2.0 * sum(corrected) - corrected[0]
    tau_int = cw / (2.0 * corrected[0])
    return mean, float(np.sqrt(max(cw, 0.0) / n)), float(tau_int), W


def _x0_unnormalised(alpha, w):
    """Integral of sqrt(1-t^2) exp(alpha (t-1)) dt over [-1, w], vectorised."""
    alpha = np.asarray(alpha, dtype=np.float64)
    w = np.clip(np.asarray(w, dtype=np.float64), -1.0, 1.0)
    alpha, w = np.broadcast_arrays(alpha, w)
    th_lo = np.arccos(w)                          # t = cos(theta), theta in [th_lo, pi]
    half = 0.5 * (np.pi - th_lo)
    mid = 0.5 * (np.pi + th_lo)
    th = mid[..., None] + half[..., None] * _GL_X
    f = np.sin(th) ** 2 * np.exp(alpha[..., None] * (np.cos(th) - 1.0))
    return (f * _GL_W).sum(-1) * half


def x0_cdf(alpha, w):
    """P(w0 <= w) for w0 with density ~ sqrt(1-w0^2) exp(alpha w0) on [-1,1]."""
    return _x0_unnormalised(alpha, w) / _x0_unnormalised(alpha, np.ones_like(np.asarray(w, float)))


def x0_norm_scaled(alpha):
    """Integral of sqrt(1-t^2) exp(alpha (t-1)) over [-1, 1] by quadrature."""
    return _x0_unnormalised(alpha, np.ones_like(np.asarray(alpha, float)))


def haar_a0_cdf(x):
    """P(a0 <= x) for a Haar-random SU(2) element: density (2/pi) sqrt(1-x^2)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return 0.5 + (x * np.sqrt(1.0 - x * x) + np.arcsin(x)) / np.pi
