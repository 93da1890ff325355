"""Statistics used by the statistical pins and the FP32-versus-FP64 checks
(test infrastructure: nothing here comes from the package under test).

- blocking_error: the error of the mean of an autocorrelated series by
  blocking (Flyvbjerg and Petersen, J. Chem. Phys. 91 (1989) 461): block
  means over blocks of 2^l samples, the standard error of the mean at every
  level that still has at least 32 blocks, and the largest of them (the
  plateau for a series much longer than its autocorrelation time).  A
  different method from the package's Gamma method, written separately;
  pinned in tests/test_stats.py by the closed form for an AR(1) process.
- x0_cdf: the exact conditional distribution function of w0 = (1/2)Tr(W)
  when W has density ~ exp(alpha w0) with respect to Haar measure on SU(2),
  i.e. w0 has density ~ sqrt(1 - w0^2) exp(alpha w0) on [-1, 1].  Computed
  by Gauss-Legendre quadrature in the angle w0 = cos(theta), where the
  integrand sin^2(theta) exp(alpha (cos(theta) - 1)) is smooth.
- haar_a0_cdf: the alpha = 0 case in closed form.
"""
import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


def blocking_error(a, min_blocks=32):
    """Return (mean, error, tau_int, levels) of the series a by blocking;
    tau_int = (error / naive error)^2 / 2, levels = the blocking levels used."""
    a = np.asarray(a, dtype=np.float64)
    mean = float(a.mean())
    n = a.size
    if n < 2:
        return mean, 0.0, 0.5, 0
    naive = float(a.std(ddof=1) / np.sqrt(n))
    x = a.copy()
    err = naive
    level = 0
    while x.size >= 2 * min_blocks:
        m = x.size // 2
        x = 0.5 * (x[:2 * m:2] + x[1:2 * m:2])
        level += 1
        err = max(err, float(x.std(ddof=1) / np.sqrt(x.size)))
    tau = 0.5 * (err / naive) ** 2 if naive > 0 else 0.5
    return mean, err, tau, level


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
