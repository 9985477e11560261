"""The GEMM epilogue's reduction of an INT32 product entry to its symmetric
residue modulo an odd p (two fmas against 1.5 2^52 and an integer add,
residue_sym_i32 in the library's header), built for the host and compared
with integer division for every odd p < 256 (CPU only; the cases are listed
in the driver's header)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_residue_sym_matches_integer_division():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    try:
        exe = os.path.join(d, "residue_host_driver")
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                               "-ffp-contract=off",
                               "-I", os.path.join(ROOT, "paper_2606_29129_amd", "csrc"),
                               os.path.join(ROOT, "tests", "residue_host_driver.cpp"), "-o", exe],
                              stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        lines = out.stdout.split()
        cases, bad = int(lines[-2]), int(lines[-1])
        assert out.returncode == 0 and bad == 0, out.stdout
        assert cases > 127 * 300000
    finally:
        shutil.rmtree(d, ignore_errors=True)
