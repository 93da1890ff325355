"""Finite-temperature analysis of the Polyakov-loop outputs (paper, section
"Finite Temperature", eqs. (1)-(3) and the fits that follow them).

Consumes what the GPU path records per sweep -- the spatial mean L of the
Polyakov loop (L(x) = (1/2) Tr of the ordered product of temporal links) and
the on-axis correlator C(r) = <L(x) L(x + r e_i)> -- and turns them into:

- the renormalised Polyakov loop <L^r> = Z(g^2)^Nt <|L|>, eq. (2), with
  Z(g^2) = exp(A g^2 + B g^4) and g^2 = 4/beta (the SU(2) Wilson action);
  A = 0.0637, B = 0.0731 are the paper's fitted values (stated valid for
  g^2 < 1.3);
- the procedure that gives Z(g^2) (the paper follows the iterative
  renormalisation of Gupta, Huebner and Kaczmarek, seeded by zero-
  temperature static potentials): a seed Z at one coupling from matching
  the bare free energy at short distance to the renormalised zero-
  temperature potential (the self energy of the two static charges is the
  only difference between them there), its transfer to other couplings
  through lattices of different Nt at the same temperature (where the
  renormalised loops must agree), and the fit of ln Z = A g^2 + B g^4;
- the colour-averaged free energy of a static pair, eq. (3): with L
  normalised by 1/2, (1/4)<Tr L Tr L^+> equals C(r), so
  F_avg(r)/T = -ln C(r) + const; the paper's shift F -> F - T ln 4 is
  applied and the undetermined constant set to zero, so
  F_avg(r)/T = -ln C(r) - ln 4.  In lattice units (T = 1/(a Nt))
  a F_avg(r) = (F_avg/T) / Nt;
- the string tension sigma(T) from the weighted fit
  a F_avg(r) = a0 - a1/r + sigma r (linear in a0, a1, sigma);
- the two ansaetze the paper fits to sigma(T):
  a sqrt(1 - b (T/Tc)^2) and a (Tc - T)^nu [1 + b sqrt(Tc - T)] (nu fixed,
  0.63 by default), with T in units of Tc.

Errors of nonlinear functions of means (the logarithm, the fit) come from
the jackknife over blocks of consecutive sweeps.  This is host-side
post-processing of the kernels' outputs; it launches nothing.
"""
import numpy as np

PAPER_Z_A = 0.0637
PAPER_Z_B = 0.0731


def renormalization_z(beta, A=PAPER_Z_A, B=PAPER_Z_B):
    """Z(g^2) = exp(A g^2 + B g^4) with g^2 = 4/beta (eq. (2))."""
    g2 = 4.0 / np.asarray(beta, dtype=np.float64)
    return np.exp(A * g2 + B * g2 * g2)


def renormalized_polyakov(L, beta, nt, A=PAPER_Z_A, B=PAPER_Z_B):
    """<L^r> = Z(g^2)^Nt <L> (eq. (2)); L may be a mean or an array of means."""
    return renormalization_z(beta, A, B) ** int(nt) * np.asarray(L, dtype=np.float64)


def z_from_short_distance(r, corr, nt, v_ren, r_max):
    """Seed of the renormalisation: ln Z at one coupling from the bare
    correlator C(r) of a lattice with Nt time slices and the renormalised
    zero-temperature potential a V(r) (lattice units) at the same coupling.

    With L^r = Z^Nt L the correlator renormalises as C^r = Z^(2 Nt) C, so
    a F^r(r) = -(1/Nt) ln C^r(r) = a F(r) - 2 ln Z.  At distances well below
    1/T the free energy is the zero-temperature potential, so over
    r <= r_max:  ln Z = mean of (a F(r) - a V(r)) / 2.  Returns (ln Z, the
    spread of the per-r values, which vanishes when the match holds)."""
    r = np.asarray(r, dtype=np.float64)
    aF = -np.log(np.asarray(corr, dtype=np.float64)) / float(nt)
    d = (aF - np.asarray(v_ren, dtype=np.float64)) / 2.0
    sel = r <= r_max
    if not np.any(sel):
        raise ValueError("no separation at or below r_max")
    return float(d[sel].mean()), float(d[sel].std())


def z_transfer(ln_z_ref, loop_ref, nt_ref, loop_new, nt_new):
    """Carry ln Z from a coupling where it is known to another one through
    two lattices at the same temperature: (Nt_ref, beta_ref) with bare loop
    loop_ref and (Nt_new, beta_new) with loop_new.  Equal renormalised loops,
    Z_ref^Nt_ref L_ref = Z_new^Nt_new L_new (eq. (2)), give
    ln Z_new = (Nt_ref ln Z_ref + ln L_ref - ln L_new) / Nt_new."""
    return (nt_ref * ln_z_ref + np.log(loop_ref) - np.log(loop_new)) / float(nt_new)


def fit_z(g2, ln_z, d_ln_z=None):
    """Weighted least squares of ln Z(g^2) = A g^2 + B g^4 (the form the
    paper fits).  Returns ((A, B), covariance, chi2/dof)."""
    g2 = np.asarray(g2, dtype=np.float64)
    y = np.asarray(ln_z, dtype=np.float64)
    w = np.ones_like(y) if d_ln_z is None else 1.0 / np.asarray(d_ln_z, dtype=np.float64) ** 2
    X = np.stack([g2, g2 * g2], axis=1)
    XtW = X.T * w
    cov = np.linalg.inv(XtW @ X)
    p = cov @ (XtW @ y)
    res = y - X @ p
    chi2 = float((w * res * res).sum()) / max(1, len(y) - 2)
    return p, cov, chi2


def renormalisation_chain(seed, steps):
    """The iterative procedure: seed = (g2, ln Z) at the starting coupling;
    steps = [(g2_ref, g2_new, loop_ref, nt_ref, loop_new, nt_new), ...], each
    a pair of lattices at one temperature whose reference coupling already
    has ln Z (the seed or an earlier step).  Returns {g2: ln Z}."""
    known = {float(seed[0]): float(seed[1])}
    for g2_ref, g2_new, loop_ref, nt_ref, loop_new, nt_new in steps:
        if float(g2_ref) not in known:
            raise ValueError(f"no ln Z yet at g^2 = {g2_ref}")
        known[float(g2_new)] = float(z_transfer(known[float(g2_ref)], loop_ref, nt_ref, loop_new, nt_new))
    return known


def jackknife_blocks(samples, n_blocks):
    """Leave-one-block-out means of `samples` (first axis = sweeps), blocks of
    equal length (a tail that does not fill a block is dropped)."""
    x = np.asarray(samples, dtype=np.float64)
    m = (x.shape[0] // n_blocks) * n_blocks
    if m == 0:
        raise ValueError("fewer samples than blocks")
    blocks = x[:m].reshape((n_blocks, m // n_blocks) + x.shape[1:]).mean(axis=1)
    total = blocks.sum(axis=0)
    return (total[None, ...] - blocks) / (n_blocks - 1)


def jackknife(fn, samples, n_blocks=20):
    """Estimate and jackknife error of fn(mean of samples)."""
    x = np.asarray(samples, dtype=np.float64)
    est = np.asarray(fn(x.mean(axis=0)), dtype=np.float64)
    loo = np.array([np.asarray(fn(b), dtype=np.float64) for b in jackknife_blocks(x, n_blocks)])
    k = loo.shape[0]
    err = np.sqrt((k - 1) / k * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))
    return est, err


def free_energy_over_t(corr):
    """F_avg(r)/T = -ln C(r) - ln 4 (eq. (3) with the paper's T ln 4 shift and
    the additive constant set to zero).  corr: C(r) for r = 1..R."""
    c = np.asarray(corr, dtype=np.float64)
    return -np.log(c) - np.log(4.0)


def free_energy_lattice(corr, nt):
    """a F_avg(r) = (F_avg/T) / Nt, since a T = 1/Nt."""
    return free_energy_over_t(corr) / float(nt)


def fit_string_tension(r, F, dF=None):
    """Weighted least squares of F(r) = a0 - a1/r + sigma r.

    Returns (params [a0, a1, sigma], covariance, chi2/dof).  The model is
    linear in its parameters, so the fit is exact linear algebra."""
    r = np.asarray(r, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    w = np.ones_like(F) if dF is None else 1.0 / np.asarray(dF, dtype=np.float64) ** 2
    X = np.stack([np.ones_like(r), -1.0 / r, r], axis=1)
    XtW = X.T * w
    cov = np.linalg.inv(XtW @ X)
    p = cov @ (XtW @ F)
    res = F - X @ p
    dof = max(1, len(F) - 3)
    chi2 = float((w * res * res).sum()) / dof
    return p, cov, chi2


def string_tension(corr_samples, nt, rmin=1, rmax=None, n_blocks=20):
    """sigma (lattice units) and its jackknife error from per-sweep
    correlators corr_samples[sweep, r-1], fitting r in [rmin, rmax]."""
    c = np.asarray(corr_samples, dtype=np.float64)
    R = c.shape[1]
    rmax = R if rmax is None else rmax
    r = np.arange(rmin, rmax + 1, dtype=np.float64)
    sel = slice(rmin - 1, rmax)
    # errors of F(r) for the weights, then the jackknife of the weighted fit
    F_est, F_err = jackknife(lambda cm: free_energy_lattice(cm[sel], nt), c, n_blocks)

    def weighted(cmean):
        return fit_string_tension(r, free_energy_lattice(cmean[sel], nt), F_err)[0]

    p, perr = jackknife(weighted, c, n_blocks)
    return p, perr, (r, F_est, F_err)


def sigma_ansatz_sqrt(t, a, b):
    """a sqrt(1 - b t^2), t = T/Tc."""
    return a * np.sqrt(np.maximum(0.0, 1.0 - b * np.asarray(t) ** 2))


def sigma_ansatz_critical(t, a, b, nu=0.63):
    """a (1 - t)^nu [1 + b sqrt(1 - t)], t = T/Tc (Tc = 1)."""
    d = np.maximum(0.0, 1.0 - np.asarray(t))
    return a * d ** nu * (1.0 + b * np.sqrt(d))


def fit_sigma_of_t(t, sigma, dsigma, ansatz="sqrt", nu=0.63, p0=None):
    """Fit sigma(T/Tc) with one of the paper's two ansaetze; returns
    (params [a, b], errors, chi2/dof)."""
    from scipy.optimize import curve_fit
    t = np.asarray(t, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    ds = np.asarray(dsigma, dtype=np.float64)
    if ansatz == "sqrt":
        f = sigma_ansatz_sqrt
        p0 = p0 or (float(s.max()), 1.0)
    elif ansatz == "critical":
        def f(x, a, b):
            return sigma_ansatz_critical(x, a, b, nu)
        p0 = p0 or (float(s.max()), 0.0)
    else:
        raise ValueError("ansatz must be 'sqrt' or 'critical'")
    p, cov = curve_fit(f, t, s, p0=p0, sigma=ds, absolute_sigma=True, maxfev=20000)
    res = (s - f(t, *p)) / ds
    chi2 = float((res * res).sum()) / max(1, len(t) - 2)
    return p, np.sqrt(np.diag(cov)), chi2
