"""Statistics used by the statistical pins and the FP32-versus-FP64 checks.

- gamma_method: error of a Monte Carlo mean with its integrated
  autocorrelation time, by the Gamma method of U. Wolff, "Monte Carlo errors
  with less errors", Comput. Phys. Commun. 156 (2004) 143, with the automatic
  summation window (S = 1.5) and the bias correction described there.
- x0_cdf: the exact conditional distribution function of w0 = (1/2)Tr(W)
  when W has density ~ exp(alpha w0) with respect to Haar measure on SU(2),
  i.e. w0 has density ~ sqrt(1 - w0^2) exp(alpha w0) on [-1, 1].  Computed
  by Gauss-Legendre quadrature in the angle w0 = cos(theta), where the
  integrand sin^2(theta) exp(alpha (cos(theta) - 1)) is smooth.
- haar_a0_cdf: the alpha = 0 case in closed form.
"""
import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


def gamma_method(a, S=1.5):
    """Return (mean, error, tau_int, window) of the series a."""
    a = np.asarray(a, dtype=np.float64)
    N = a.size
    mean = a.mean()
    d = a - mean
    gamma0 = np.dot(d, d) / N
    if gamma0 == 0.0:
        return mean, 0.0, 0.5, 0
    tmax = N // 2
    gam = np.empty(tmax + 1)
    gam[0] = gamma0
    for t in range(1, tmax + 1):
        gam[t] = np.dot(d[:N - t], d[t:]) / (N - t)
    window = tmax
    tau_w = 0.5
    for W in range(1, tmax + 1):
        tau_w = 0.5 + gam[1:W + 1].sum() / gamma0
        if tau_w <= 0.5:
            window = W
            break
        tau = S / np.log((2 * tau_w + 1) / (2 * tau_w - 1))
        g = np.exp(-W / tau) - tau / np.sqrt(W * N)
        if g < 0:
            window = W
            break
    # bias correction of the estimated Gamma(0) and tau_int
    c_total = gamma0 + 2 * gam[1:window + 1].sum()
    c_total *= 1.0 + (2 * window + 1) / N
    tau_int = max(c_total / (2 * gamma0), 0.5)
    err = np.sqrt(max(c_total, 0.0) / N)
    return mean, err, tau_int, window


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
