"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/oracle_sanitized.c calls every entry point of oracle/su2_oracle.c
(random numbers, algebra, geometry, starts, FP64 and single-precision heat
bath, overrelaxation, observables, gauge transformation, the learned block
move's reference) on small and ragged lattices.  Built with
-fsanitize=address,undefined and no recovery, any out-of-bounds access,
use of freed memory, leak or undefined arithmetic ends the run with an
error; the values it prints must equal those of the regular (optimised,
OpenMP) build of the oracle.  Host only.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized_run(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("osan") / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-Werror",
           "-I" + os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "native", "oracle_sanitized.c"),
           os.path.join(ROOT, "oracle", "su2_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = {}
    for line in r.stdout.splitlines():
        name, *vals = line.split()
        out[name] = vals
    return r, out


def test_oracle_is_clean_under_sanitizers(sanitized_run):
    r, out = sanitized_run
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "block_plaquette" in out and "colour" in out            # ran to the end


def test_sanitized_build_agrees_with_regular_build(sanitized_run):
    _, out = sanitized_run
    n, seed, beta, lid = (6, 4, 10, 8), 1234, 2.3, 3
    U = oracle.init_hot(n, seed, lattice_id=lid)
    for s in range(3):
        assert oracle.heatbath_sweep(n, U, beta, seed, s, lattice_id=lid) == 0
        oracle.overrelax_sweep(n, U)
    for mu in range(4):
        for p in range(2):
            oracle.heatbath_halfsweep(n, U, beta, seed, 7, mu, p, lattice_id=lid)
            oracle.overrelax_halfsweep(n, U, mu, p)
    P, planes = oracle.plaquette(n, U)
    lm, la = oracle.polyakov(n, U)
    C = oracle.polyakov_corr(n, U)
    assert int(out["ragged_flags"][0]) == 0
    assert abs(float(out["ragged_plaquette"][0]) - P) <= 1e-12
    assert abs(float(out["ragged_plane5"][0]) - planes[5]) <= 1e-12
    assert abs(float(out["ragged_poly_mean"][0]) - lm) <= 1e-12
    assert abs(float(out["ragged_poly_abs"][0]) - la) <= 1e-12
    assert abs(float(out["ragged_corr_last"][0]) - C[-1]) <= 1e-12
    # gauge invariance holds in the sanitized build too
    assert abs(float(out["ragged_plaquette_gauge"][0]) - P) <= 1e-13
    # the single-precision step
    V = oracle.init_hot(n, 99)
    V = V.astype(np.float32).astype(np.float64)
    for mu in range(4):
        for p in range(2):
            assert oracle.heatbath_halfsweep_f32(n, V, beta, 99, 1, mu, p) == 0
    assert abs(float(out["f32_plaquette"][0]) - oracle.plaquette(n, V)[0]) <= 1e-12
