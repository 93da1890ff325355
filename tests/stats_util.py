"""Statistics used by the statistical pins and the FP32-versus-FP64 checks.

- gamma_method: re-exported from paper_1104_5432_amd.stats (Wolff's Gamma
  method), pinned in tests/test_stats.py.
- x0_cdf: the exact conditional distribution function of w0 = (1/2)Tr(W)
  when W has density ~ exp(alpha w0) with respect to Haar measure on SU(2),
  i.e. w0 has density ~ sqrt(1 - w0^2) exp(alpha w0) on [-1, 1].  Computed
  by Gauss-Legendre quadrature in the angle w0 = cos(theta), where the
  integrand sin^2(theta) exp(alpha (cos(theta) - 1)) is smooth.
- haar_a0_cdf: the alpha = 0 case in closed form.
"""
import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(96)


from paper_1104_5432_amd.stats import gamma_method  # noqa: E402,F401  (pinned in test_stats.py)


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
