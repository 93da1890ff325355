import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: statistical test taking more than a few seconds")
    # the package loads libsu2.so on import; build it once if nothing is built
    # (build.py is loaded by path: importing it through the package would load
    # the library first)
    import importlib.util
    build_py = os.path.join(ROOT, "paper_1104_5432_amd", "build.py")
    if not os.path.exists(build_py):    # a tree holding only the oracle and its tests
        return
    spec = importlib.util.spec_from_file_location("_su2_build", build_py)
    hip_build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(hip_build)
    if not os.path.exists(hip_build.LIB):
        hip_build.build()
