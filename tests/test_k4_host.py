"""K4's per-entry arithmetic (the exact CRT of Step 3 and the correctly
rounded unscaling of Step 4) built for the host from the library's own
header, against the oracle (CPU only).

Each case is a value C'' with |C''| < P/2, given to the host build as its
INT8 residues (as K3 writes them); the oracle's expected output is
RN(C'' 2^-E) in binary64 and binary32, by Python integer arithmetic.  The
values are chosen to reach every branch of the reconstruction and rounding:
random magnitudes of every length, exact ties and near-ties at the 53- and
24-bit rounding positions (with and without bits far below), values next to
+-P/2 (the quotient correction), zero and tiny values, and exponents that put
the result near the smallest normal number, deep in the subnormal range,
near overflow and beyond."""
import os
import random
import shutil
import struct
import subprocess
import tempfile

import pytest

from oracle import constants, fp, ozaki2 as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "k4_host_driver")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2606_29129_amd", "csrc"),
                           os.path.join(ROOT, "tests", "k4_host_driver.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def _values(rng, P, count):
    """C'' values (|C''| < P/2) of the kinds listed in the module docstring."""
    half = P // 2
    nbits = half.bit_length()
    out = [0, 1, -1, half - 1, -(half - 1)]
    for _ in range(count):
        kind = rng.randrange(8)
        nb = rng.randint(1, nbits)
        v = rng.getrandbits(nb) | (1 << (nb - 1))
        if kind in (1, 2, 3):                 # tie at 53 or 24 bits, maybe a sticky bit
            prec = 24 if kind == 3 else 53
            cut = nb - 1 - prec               # position of the rounding bit
            if cut >= 0:
                v = (v >> (cut + 1) << (cut + 1)) | (1 << cut)
                if kind == 2 and cut > 0:
                    v |= 1 << rng.randrange(cut)
        elif kind == 4:                       # one below a tie
            prec = rng.choice((24, 53))
            cut = nb - 1 - prec
            if cut >= 1:
                v = (v >> (cut + 1) << (cut + 1)) | ((1 << cut) - 1)
        elif kind == 5:                       # next to +-P/2
            v = half - rng.randint(1, 1 << 20)
        elif kind == 6:                       # a few bits spread over the slices
            v = 1 << (nb - 1)
            for _ in range(3):
                v |= 1 << rng.randrange(nb)
        if v >= half or v <= 0:
            continue
        out.append(-v if rng.random() < 0.5 else v)
    return out


def _exponents(rng, v):
    """Scale exponents E around the interesting ranges for |v|'s leading bit."""
    L = abs(v).bit_length() - 1 if v else 0
    return [rng.randint(-100, 100),
            L + 1022 - rng.randint(0, 60), L + 1022, L + 1023, L + 1074 + rng.randint(-2, 2),
            L - 1023 + rng.randint(-1, 1),
            L + 126 - rng.randint(0, 30), L + 126, L + 149 + rng.randint(-2, 2),
            L - 127 + rng.randint(-1, 1)]


@pytest.mark.parametrize("N", [2, 4, 5, 9, 10, 14, 15, 17, 20])
def test_crt_unscale_host_build_matches_oracle(driver, N):
    p, P, _, _ = constants.step1(N)
    rng = random.Random(1000 + N)
    cases = []
    for v in _values(rng, P, 400):
        U = [ref.residue(v, pt) for pt in p]
        for E in _exponents(rng, v):
            cases.append((v, E, U))
    text = "".join(f"{N} {E} " + " ".join(map(str, U)) + "\n" for v, E, U in cases)
    res = subprocess.run([driver], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.split()
    assert len(lines) == 2 * len(cases)
    bad = []
    for i, (v, E, U) in enumerate(cases):
        # the residues determine C'' (|C''| < P/2): the oracle's CRT
        Cp = sum(Pi * qi * u for Pi, qi, u in zip(*constants.step1(N)[2:], U))
        assert ref.rmod(Cp, P) == v
        want64 = struct.unpack("<Q", struct.pack("<d", fp.round_dyadic(v, -E, fp.BINARY64)))[0]
        want32 = struct.unpack("<I", struct.pack("<f", fp.round_dyadic(v, -E, fp.BINARY32)))[0]
        got64, got32 = int(lines[2 * i], 16), int(lines[2 * i + 1], 16)
        if (got64, got32) != (want64, want32):
            bad.append((v, E, hex(got64), hex(want64), hex(got32), hex(want32)))
    assert not bad, bad[:5]
