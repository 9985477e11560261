"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, validates arguments before touching the device, and
computes the same Step 1 constants as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import constants
from paper_2606_29129_amd import ozaki2 as oz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ozaki2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ozaki2_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(oz.LIB_PATH)
    names = _declared()
    assert "ozaki2_dgemm" in names and "ozaki2_sgemm" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps each of them under the same name
    for name in names:
        assert callable(getattr(oz, name)), name


@pytest.mark.parametrize("args,code", [
    ((-1, 1, 1, 1, 1, 1, 1, 1, 1, 14, 0), -1),
    ((1, -1, 1, 1, 1, 1, 1, 1, 1, 14, 0), -2),
    ((1, 1, -1, 1, 1, 1, 1, 1, 1, 14, 0), -3),
    ((4, 4, 4, 0, 4, 1, 4, 1, 4, 14, 0), -4),
    ((4, 4, 4, 1, 3, 1, 4, 1, 4, 14, 0), -5),
    ((4, 4, 4, 1, 4, 0, 4, 1, 4, 14, 0), -6),
    ((4, 4, 4, 1, 4, 1, 3, 1, 4, 14, 0), -7),
    ((4, 4, 4, 1, 4, 1, 4, 0, 4, 14, 0), -8),
    ((4, 4, 4, 1, 4, 1, 4, 1, 3, 14, 0), -9),
    ((4, 4, 4, 1, 4, 1, 4, 1, 4, 1, 0), -10),
    ((4, 4, 4, 1, 4, 1, 4, 1, 4, 21, 0), -10),
    ((4, 4, 4, 1, 4, 1, 4, 1, 4, 14, 4), -11),
    ((4, 4, 2**22 + 1, 1, 4, 1, 2**22 + 1, 1, 4, 14, 0), 1),    # OZ2_K_MAX
    ((4, 4, 2**18 + 1, 1, 4, 1, 2**18 + 1, 1, 4, 14, 2), 1),    # accurate mode
])
def test_argument_errors_are_reported_without_device_work(args, code):
    assert oz.ozaki2_dgemm(*args) == code
    assert oz.ozaki2_sgemm(*args) == code
    assert oz.ozaki2_dgemm_noalloc(*args) == code


def test_quick_returns_need_no_device():
    # m = 0 or n = 0: nothing to compute; only the operand with elements
    # needs a (never dereferenced) pointer.
    assert oz.ozaki2_dgemm(0, 5, 5, 0, 1, 8, 5, 0, 1, 14, 0) == 0
    assert oz.ozaki2_dgemm(5, 0, 5, 8, 5, 0, 5, 0, 5, 14, 0) == 0


def test_status_strings():
    for c in (-3, 0, 1, 2, 3, 4, 5, 99):
        assert isinstance(oz.ozaki2_status_string(c), str)
    v = oz.ozaki2_version()
    assert "kc=64" in v and "gfx950" in v


@pytest.mark.parametrize("N", range(2, 21))
def test_library_constants_match_oracle(N):
    c = oz.ozaki2_query_constants(N)
    assert c["moduli"] == list(constants.moduli(N))
    assert np.float32(c["p_prime_prop"]) == np.float32(float(constants.p_prime_prop(N)))
    assert np.float32(c["p_prime_fast"]) == np.float32(float(constants.p_prime_fast(N)))
    assert np.float32(c["delta"]) == np.float32(float(constants.delta()))
    _, P, _, _ = constants.step1(N)
    assert abs(c["log2_P"] - np.log2(float(P))) < 1e-9


def test_workspace_size_grows_with_problem():
    a = oz.ozaki2_workspace_size(256, 256, 256, 14)
    b = oz.ozaki2_workspace_size(1024, 1024, 1024, 14)
    c = oz.ozaki2_workspace_size(1024, 1024, 1024, 20)
    assert 0 < a < b < c
    assert oz.ozaki2_workspace_size(0, 10, 10, 14) == 0


def test_tile_policy_and_automatic_choice():
    """ozaki2_set_tile validates its argument; the automatic choice is
    deterministic host logic: the wide tile for large squares, the narrow one
    for n = 64."""
    assert oz.ozaki2_set_tile(7) == -1
    assert oz.ozaki2_set_tile(-1) == -1
    assert oz.ozaki2_set_tile(oz.TILE_AUTO) == 0
    assert oz.ozaki2_get_tile(16384, 16384, 16384, 14) == oz.TILE_256x256
    assert oz.ozaki2_get_tile(8192, 8192, 8192, 14) == oz.TILE_256x256
    assert oz.ozaki2_get_tile(65536, 64, 4096, 14) == oz.TILE_256x64
    for t in (oz.TILE_256x256, oz.TILE_128x128, oz.TILE_256x64):
        assert oz.ozaki2_set_tile(t) == 0
        assert oz.ozaki2_get_tile(16384, 16384, 16384, 14) == t
    assert oz.ozaki2_set_tile(oz.TILE_AUTO) == 0
    t = ctypes.c_int(0)
    lib = oz.lib()
    assert lib.ozaki2_get_tile(1, 1, 1, 1, ctypes.byref(t)) == -4
    assert lib.ozaki2_get_tile(-1, 1, 1, 14, ctypes.byref(t)) == -1
    assert lib.ozaki2_get_tile(1, 1, 1, 14, None) == -5


def test_k_limits_of_the_header():
    """The k limits: one INT8 GEMM block, the general limit, accurate mode's;
    a batch rejects k beyond one block for its problem."""
    hdr = open(os.path.join(ROOT, "include", "ozaki2.h")).read()
    vals = {k: int(v) for k, v in re.findall(r"#define (OZ2_K_\w+)\s+(\d+)", hdr)}
    assert vals == {"OZ2_K_BLOCK": 2**17, "OZ2_K_MAX": 2**22, "OZ2_K_MAX_ACCURATE": 2**18}
    # INT32 exactness of one block for odd moduli, and of the bar product
    assert 2**17 * 127**2 < 2**31 and 64 * 64 * 2**18 < 2**31
    bad = ctypes.c_int(-1)
    prob = oz.Oz2Problem(4, 4, 2**17 + 1, 8, 4, 8, 2**17 + 1, 8, 4, 14, 0)
    arr = (oz.Oz2Problem * 1)(prob)
    assert oz.lib().ozaki2_dgemm_batched(1, arr, 0, 0.0, ctypes.byref(bad)) == 1 and bad.value == 0


@pytest.mark.parametrize("args,code", [
    ((-1, 1, 1, 16, 1, 16, 1, 16, 1, 14, 0), -1),
    ((4, 4, 4, 16, 3, 16, 4, 16, 4, 14, 0), -5),
    ((4, 4, 4, 16, 4, 16, 4, 16, 4, 21, 0), -10),
    ((4, 4, 4, 16, 4, 16, 4, 16, 4, 14, 4), -11),
    ((4, 4, 4, 16, 4, 16, 4, 16, 4, 14, 2), 4),     # accurate mode: unsupported
    ((4, 4, 4, 24, 4, 16, 4, 16, 4, 14, 0), -4),    # A not aligned to a complex entry
    ((4, 4, 4, 16, 4, 40, 4, 16, 4, 14, 0), -6),
    ((4, 4, 4, 16, 4, 16, 4, 56, 4, 14, 0), -8),
    ((4, 4, 2**22 + 1, 16, 4, 16, 2**22 + 1, 16, 4, 14, 0), 1),
])
def test_complex_argument_errors_without_device_work(args, code):
    assert oz.ozaki2_zgemm(*args) == code
    if code in (-4, -6, -8):
        # binary32 pairs need 8-byte alignment only: 24, 40 and 56 are fine
        return
    assert oz.ozaki2_cgemm(*args) == code


def test_cgemm_alignment_is_one_complex64_entry():
    assert oz.ozaki2_cgemm(4, 4, 4, 20, 4, 16, 4, 16, 4, 14, 0) == -4
    assert oz.ozaki2_cgemm(0, 4, 4, 16, 1, 16, 4, 16, 1, 14, 0) == 0   # quick return


def test_complex_workspace_holds_three_components():
    r = oz.ozaki2_workspace_size(1024, 1024, 1024, 14)
    z = oz.ozaki2_zgemm_workspace_size(1024, 1024, 1024, 14)
    assert 3 * (r - 2**20) < z < 3 * r + 2**20
    assert oz.ozaki2_zgemm_workspace_size(0, 5, 5, 14) == 0
    with pytest.raises(oz.Ozaki2Error):
        oz.ozaki2_zgemm_workspace_size(8, 8, 8, 14, 2)


def _probs(shapes_N):
    out = []
    for m, n, k, N in shapes_N:
        out.append((m, n, k, 256, max(1, m), 256, max(1, k), 256, max(1, m), N))
    return out


def test_batched_workspace_size_is_a_bound_over_N():
    """Host only: the batch's workspace size grows with N, counts N = 0 as
    the maximum N (20) plus scratch for the phi estimate, is at least the sum of the single-call workspaces of
    its problems (each problem keeps its own regions), and reports argument
    errors like the batched call."""
    shapes = [(100, 70, 300), (64, 64, 64), (1500, 33, 900)]
    sz = {N: oz.ozaki2_dgemm_batched_workspace_size(_probs([s + (N,) for s in shapes]))
          for N in (8, 14, 20, 0)}
    # N = 0 plans N = 20 plus the phi estimate's scratch (two operands each)
    assert sz[8] < sz[14] < sz[20] < sz[0] <= sz[20] + 4096
    singles = sum(oz.ozaki2_workspace_size(m, n, k, 20, 0) for m, n, k in shapes)
    assert sz[20] > 0
    # single-call layouts use 256-row tiles, the batch 128: compare per problem
    # against its own 128-tile need instead of the single-call figure
    assert sz[20] >= sum(20 * ((m + 127) // 128 * 128) * ((k + 127) // 128 * 128)
                         for m, n, k in shapes)
    assert singles > 0
    # problems with nothing to compute need no workspace
    assert oz.ozaki2_dgemm_batched_workspace_size(_probs([(0, 5, 5, 14), (5, 5, 0, 14)])) == 0
    lib = oz.lib()
    b = ctypes.c_size_t(0)
    arr = oz._problem_array(_probs([(4, 4, 4, 14)]))
    assert lib.ozaki2_dgemm_batched_workspace_size(-1, arr, 0, ctypes.byref(b)) == -1
    assert lib.ozaki2_dgemm_batched_workspace_size(1, None, 0, ctypes.byref(b)) == -2
    assert lib.ozaki2_dgemm_batched_workspace_size(1, arr, 2, ctypes.byref(b)) == -3
    assert lib.ozaki2_dgemm_batched_workspace_size(1, arr, 0, None) == -4
    bad = oz._problem_array(_probs([(4, 4, 4, 21)]))
    assert lib.ozaki2_dgemm_batched_workspace_size(1, bad, 0, ctypes.byref(b)) == -10


def test_workspace_policy_values():
    assert oz.ozaki2_set_workspace_policy(2) == -1
    assert oz.ozaki2_set_workspace_policy(oz.WORKSPACE_LIBRARY) == 0
    assert oz.ozaki2_set_workspace_policy(oz.WORKSPACE_CALLER) == 0


def test_fp8_engine_flag_on_the_host():
    """OZ2_ENGINE_FP8 (16) or-ed into the mode: the workspace grows by the two
    E4M3 digit planes per modulus and operand; accurate mode with the flag is
    unsupported (4); an unknown base mode with the flag is still argument 11."""
    m, n, k, N = 300, 200, 500, 14
    base = oz.ozaki2_workspace_size(m, n, k, N, 0)
    with8 = oz.ozaki2_workspace_size(m, n, k, N, 16)
    pad = lambda x: (x + 255) // 256 * 256
    assert with8 - base >= 2 * N * (pad(m) + pad(n)) * pad(k)
    for mode in (1, 3):
        assert oz.ozaki2_workspace_size(m, n, k, N, mode | 16) > oz.ozaki2_workspace_size(m, n, k, N, mode)
    b = ctypes.c_size_t(0)
    assert oz.lib().ozaki2_workspace_size(m, n, k, N, 2 | 16, ctypes.byref(b)) == 4
    assert oz.ozaki2_dgemm(4, 4, 4, 1, 4, 1, 4, 1, 4, 14, 4 | 16) == -11
    assert oz.ozaki2_dgemm(4, 4, 4, 1, 4, 1, 4, 1, 4, 21, 16) == -10
