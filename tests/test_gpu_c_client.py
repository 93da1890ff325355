"""The C ABI on its own: tests/native/abi_client.c, a plain C program built
with gcc against include/su2.h and libsu2.so (no PyTorch, no C++), allocates
with the HIP runtime, runs a hot start and two steps of 1 heat-bath + 1
overrelaxation sweep, and prints the plaquette, the Polyakov loop and the
flags; they must equal, bitwise, what the same calls give through the
Python binding."""
import os
import shutil
import subprocess

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_5432_amd  # noqa: F401  (the library is built and loads)
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("abi") / "abi_client")
    pkg = os.path.join(ROOT, "paper_1104_5432_amd")
    subprocess.run([cc, "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
                    "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
                    os.path.join(ROOT, "tests", "native", "abi_client.c"),
                    "-L" + pkg, "-lsu2", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + pkg, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe],
                   check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c_client_matches_the_binding(client, prec):
    import paper_1104_5432_amd as su2
    n, beta, seed = (8, 8, 8, 8), 2.3, 1234
    print(f"C client {n} {prec}", flush=True)
    r = subprocess.run([client, *map(str, n), "0" if prec == "f64" else "1", repr(beta), str(seed)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = dict((ln.split()[0], ln.split()[1:]) for ln in r.stdout.splitlines())
    lat = su2.Lattice(n, prec, device="cuda")
    su2.su2_init_hot(lat, seed)
    for s in range(2):
        su2.su2_heatbath_sweep(lat, beta, seed, s)
        su2.su2_overrelax(lat, 1)
    plaq = su2.su2_plaquette(lat)
    poly, _ = su2.su2_polyakov(lat, with_corr=False)
    flags = su2.su2_get_flags(lat)
    torch.cuda.synchronize()
    assert float(out["plaquette"][0]) == plaq[0].item()
    assert float(out["polyakov"][0]) == poly[0].item() and float(out["polyakov"][1]) == poly[1].item()
    assert int(out["flags"][0]) == int(flags.item()) == 0
