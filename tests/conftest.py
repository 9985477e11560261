import ctypes
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def fenv():
    """tests/fenv_ref.c built with gcc: directed rounding done by the host
    FPU under fesetround, independent of the oracle's rational rounding."""
    d = tempfile.mkdtemp()
    so = os.path.join(d, "fenv_ref.so")
    subprocess.check_call(["gcc", "-O0", "-frounding-math", "-shared", "-fPIC",
                           os.path.join(ROOT, "tests", "fenv_ref.c"), "-o", so, "-lm"])
    lib = ctypes.CDLL(so)
    lib.ru_norm_chunked.restype = ctypes.c_double
    lib.ru_norm_chunked.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    return lib
