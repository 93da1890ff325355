"""Do the oracle's pins catch plausible mistakes?  Each case plants one
mistake in a copy of the CPU oracle (on the CPU: a dropped dagger, swapped
factors, a sign, a dropped factor, a wrong extent or constant), rebuilds it
and runs a pin (from tests/test_oracle_pins.py, or tests/test_oracle_block.py
for the block move) against the copy, which must fail an assertion.

Each case rebuilds the oracle copy and runs the pin named for it in
CATCHES (a few seconds a case; the block move's stationary-law pin ~15 s).  One plausible mistake is known to pass every pin and
is not listed: multiplying the sampled element on the other side of Vhat
(Vhat^+ W instead of W Vhat^+) gives the same conditional law, since
conjugation by Vhat preserves the Haar measure and the trace; that side is a
convention of the random-number contract, fixed by the GPU-vs-oracle
per-link parity tests instead.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTATIONS = [
    ("lower staple: dagger dropped", "or_qdag(link(U, xpm, nu), d);", "memcpy(d, link(U, xpm, nu), sizeof d);"),
    ("upper staple: factors swapped", "or_qmul(link(U, xp, nu), d, t1);", "or_qmul(d, link(U, xp, nu), t1);"),
    ("quaternion product: cross-product sign", "double r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);",
     "double r1 = a[0] * b[1] + b[0] * a[1] + (a[2] * b[3] - a[3] * b[2]);"),
    ("single precision: cos^2 -> cos", "(double)(c * c) * (double)l3", "(double)c * (double)l3"),
    ("single precision: wrong Philox word", "*ub = or_u01_f32(r[2]);", "*ub = or_u01_f32(r[1]);"),
    ("single precision: staple factors swapped", "qmul_f(a, b, t);\n        qmul_f(t, c, s);\n        for (int k = 0; k < 4; ++k)\n            V[k] += s[k];\n        int64_t xm",
     "qmul_f(b, a, t);\n        qmul_f(t, c, s);\n        for (int k = 0; k < 4; ++k)\n            V[k] += s[k];\n        int64_t xm"),
    ("Kennedy-Pendleton: cos^2 -> cos", "c * c * log(u3)", "c * log(u3)"),
    ("Kennedy-Pendleton: accept test", "u4 * u4 <= 1.0 - lam2", "u4 <= 1.0 - lam2"),
    ("Kennedy-Pendleton: x0 factor", "x0 = 1.0 - 2.0 * lam2;", "x0 = 1.0 - lam2;"),
    ("Creutz: accept test", "if (u2 * u2 <= 1.0 - t * t) {", "if (u2 <= 1.0 - t * t) {"),
    ("Creutz: exponent", "double e = exp(-2.0 * alpha);", "double e = exp(-alpha);"),
    ("direction: cos(theta)", "double cth = 2.0 * u5 - 1.0;", "double cth = u5;"),
    ("new link: no dagger on Vhat", "or_qdag(Vhat, Vd);", "memcpy(Vd, Vhat, sizeof Vd);"),
    ("overrelaxation: dagger dropped", "or_qdag(Ul, Ud);", "memcpy(Ud, Ul, sizeof Ud);"),
    ("plaquette: dagger dropped", "or_qdag(link(U, xnu, mu), c);", "memcpy(c, link(U, xnu, mu), sizeof c);"),
    ("Polyakov loop: product order", "or_qmul(P, link(U, s + vs * t, 3), T);", "or_qmul(link(U, s + vs * t, 3), P, T);"),
    ("Philox: Weyl constant", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    ("FP64 uniform: shift", "uint64_t m = w >> 12;", "uint64_t m = w >> 11;"),
    ("hot start: Box-Muller angle", "r2 * sin(2.0 * OR_PI * u4)}", "r2 * sin(2.0 * OR_PI * u3)}"),
    ("correlator: wrong extent", "int64_t sy = x + (int64_t)n[0] * ((y + r) % n[1] + (int64_t)n[1] * z);",
     "int64_t sy = x + (int64_t)n[0] * ((y + r) % n[2] + (int64_t)n[1] * z);"),
    ("beta convention", "double alpha = beta * k;", "double alpha = 0.5 * beta * k;"),
    ("gauge transformation: dagger dropped", "or_qdag(g + 4 * j, gd);", "memcpy(gd, g + 4 * j, sizeof gd);"),
]

# Mistakes in the learned block move (Metropolis-Hastings on the block
# marginal, then a heat-bath redraw of the integrated links), caught by its
# own pins (tests/test_oracle_block.py).  The move is exact for any proposal,
# so a wrong proposal coefficient changes only its acceptance; the pin of
# the coefficients as slopes of the marginal catches it.
BLOCK_MUTATIONS = [
    ("block move: proposal terms swapped", "half_tr(T, M) - half_tr(Tn, M);", "half_tr(Tn, M) - half_tr(T, M);"),
    ("block move: marginal dropped", "double logr = block_log_marginal(beta, S, Tn) - block_log_marginal(beta, S, T) +",
     "double logr = 0.0 +"),
    ("block move: accept test reversed", "if (log(ua) < logr) {", "if (log(ua) > logr) {"),
    ("block move: redraw at beta = 1", "double Vb[4] = {beta * V[0], beta * V[1], beta * V[2], beta * V[3]};",
     "double Vb[4] = {V[0], V[1], V[2], V[3]};"),
    ("block move: no redraw", "memcpy(U + (o * 4 + 3) * 4, Un, sizeof Un);", ";"),
    ("block move: proposal coefficient", "or_bessel_ratio(a0) / sqrt(s * s + 1.0) * exp(y[d])",
     "or_bessel_ratio(a0) * sqrt(s * s + 1.0) * exp(y[d])"),
]

# The pin that catches each mistake (others may catch it too).
CATCHES = {
    'lower staple: dagger dropped': 'test_staple_gives_local_action_change',
    'upper staple: factors swapped': 'test_staple_gives_local_action_change',
    'quaternion product: cross-product sign': 'test_quaternion_algebra_matches_matrices',
    'single precision: cos^2 -> cos': 'test_single_precision_heatbath_law_and_agreement',
    'single precision: wrong Philox word': 'test_single_precision_heatbath_law_and_agreement',
    'single precision: staple factors swapped': 'test_single_precision_heatbath_law_and_agreement',
    'Kennedy-Pendleton: cos^2 -> cos': 'test_single_link_sampler_law',
    'Kennedy-Pendleton: accept test': 'test_single_link_sampler_law',
    'Kennedy-Pendleton: x0 factor': 'test_single_link_sampler_law',
    'Creutz: accept test': 'test_single_link_sampler_law',
    'Creutz: exponent': 'test_single_link_sampler_law',
    'direction: cos(theta)': 'test_single_link_sampler_law',
    'new link: no dagger on Vhat': 'test_heatbath_pit_at_equilibrium',
    'overrelaxation: dagger dropped': 'test_overrelaxation_invariants',
    'plaquette: dagger dropped': 'test_plaquette_constant_field_closed_form',
    'Polyakov loop: product order': 'test_gauge_invariance',
    'Philox: Weyl constant': 'test_philox_matches_independent_engine',
    'FP64 uniform: shift': 'test_u01_edges',
    'hot start: Box-Muller angle': 'test_hot_start_is_haar',
    'correlator: wrong extent': 'test_polyakov_closed_forms',
    'beta convention': 'test_strong_coupling_plaquette',
    'gauge transformation: dagger dropped': 'test_gauge_invariance',
    'block move: proposal terms swapped': 'test_block_move_samples_the_marginal',
    'block move: marginal dropped': 'test_block_move_samples_the_marginal',
    'block move: accept test reversed': 'test_block_move_samples_the_marginal',
    'block move: redraw at beta = 1': 'test_block_move_redraws_the_neighbours_from_their_conditional_law',
    'block move: no redraw': 'test_block_move_redraws_the_neighbours_from_their_conditional_law',
    'block move: proposal coefficient': 'test_block_proposal_is_the_slope_of_the_marginal',
}

CASES = ([m + ("test_oracle_pins.py",) for m in MUTATIONS]
         + [m + ("test_oracle_block.py",) for m in BLOCK_MUTATIONS])


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new,pins", CASES, ids=[c[0] for c in CASES])
def test_pins_catch_planted_mistake(name, old, new, pins, tmp_path):
    # a tree of its own per case, so that cases can run in parallel workers
    tree = str(tmp_path / "mutant")
    os.makedirs(tree)
    ign = shutil.ignore_patterns("*.so", "__pycache__", "_build")
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tree, "oracle"), ignore=ign)
    shutil.copytree(HERE, os.path.join(tree, "tests"), ignore=ign)
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tree)
    src_path = os.path.join(tree, "oracle", "su2_oracle.c")
    src = open(src_path).read()
    # the first occurrence: the sampler steps of the heat bath come before
    # their single-precision twin and the block move's neighbour redraw
    assert old in src, "mutation anchor not found: " + name
    open(src_path, "w").write(src.replace(old, new, 1))
    # the mutant must build: a failure to compile is not a caught mistake
    b = subprocess.run([sys.executable, os.path.join("oracle", "build.py")], cwd=tree, capture_output=True,
                       text=True, timeout=300)
    assert b.returncode == 0, f"mutant does not build: {name}\n{b.stderr[-2000:]}"
    # the copy's oracle and tests come first on the path (the working
    # directory); anything else resolves to this repository
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join("tests", pins) + "::" + CATCHES[name]],
                       cwd=tree, capture_output=True, text=True, timeout=900, env=env)
    shutil.rmtree(tree)
    summary = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    assert r.returncode == 1 and " failed" in summary and "error" not in summary, \
        f"the pins did not catch: {name}\n{r.stdout[-2000:]}"
