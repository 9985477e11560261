"""The residue arithmetic around 1.5 2^52, built for the host from the
library's headers (CPU only; the cases are listed in the driver's header):
the GEMM epilogue's reduction of an INT32 product entry to its symmetric
residue modulo an odd p (residue_sym_i32: two fmas and an integer add), and
K2's residue of a truncated scaled entry from its 40-bit limbs (residue_odd:
two fmas and an add after the limb combination), each compared with integer
division for every odd p < 256."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_residues_match_integer_division():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    try:
        exe = os.path.join(d, "residue_host_driver")
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                               "-ffp-contract=off",
                               "-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(ROOT, "paper_2606_29129_amd", "csrc"),
                               os.path.join(ROOT, "tests", "residue_host_driver.cpp"), "-o", exe],
                              stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        lines = out.stdout.split()
        cases, bad = int(lines[-2]), int(lines[-1])
        assert out.returncode == 0 and bad == 0, out.stdout
        assert cases > 127 * 380000
    finally:
        shutil.rmtree(d, ignore_errors=True)
