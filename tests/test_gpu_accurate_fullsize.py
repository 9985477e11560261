"""GPU parity of accurate mode (Section 2.3) at m = n = k = 8192, N = 14,
entries (rand - 0.5) exp(randn), seed 0, launched as bench.py launches it
(column-major operands, library stream, caller workspace).

Accurate mode's exponents depend on the whole bar product: the exponent of
row i needs the largest entry of row i of Cbar = Abar Bbar, and that of
column j the largest entry of column j.  For sampled rows and columns the
check takes the oracle's first step in array form (``scaling.accurate_bars``)
over all of A and B, forms the needed row and column of Cbar with a binary64
matrix-vector product (exact: the entries are integers below 2^25), takes
the oracle's final exponent step, and computes the sampled entries one by
one (``ozaki2.entry``); they must match the GPU bit for bit.  Every entry of
C is also checked against the componentwise bound 2^-40 (|A||B|)_ij around
native FP64.
"""
import numpy as np
import pytest

from oracle import constants, ozaki2 as ref, scaling
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

SIZE, N, PHI, SEED, MODE = 8192, 14, 1.0, 0, 2


@pytest.fixture(scope="module")
def accurate_problem():
    dev = torch.device("cuda:0")
    A = inputs.ozaki_matrix_torch(SIZE, SIZE, PHI, SEED, 0, dev)
    B = inputs.ozaki_matrix_torch(SIZE, SIZE, PHI, SEED, 1, dev)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((SIZE, SIZE), dtype=torch.float64, device=dev)
    ws_bytes = oz.ozaki2_workspace_size(SIZE, SIZE, SIZE, N, MODE)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    assert oz.ozaki2_set_workspace(ws_ptr, ws_bytes) == 0
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    print(f"accurate mode {SIZE}^3 N={N} phi={PHI}", flush=True)
    rc = oz.ozaki2_dgemm(SIZE, SIZE, SIZE, A_cm, SIZE, B_cm, SIZE, C_cm, SIZE, N, MODE)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    assert oz.ozaki2_set_workspace(None, 0) == 0
    del ws, A_cm, B_cm
    yield A, B, C_cm
    del A, B, C_cm
    torch.cuda.empty_cache()


def test_accurate_sampled_entries_bit_exact(accurate_problem):
    A, B, C_cm = accurate_problem
    Ah = A.cpu().numpy()
    Bh = B.cpu().numpy()
    e1A, nzA, barA = scaling.accurate_bars(Ah)          # rows of A
    e1B, nzB, barBt = scaling.accurate_bars(Bh.T)       # columns of B
    Af = barA.astype(np.float64)
    Bf = np.ascontiguousarray(barBt.T.astype(np.float64))   # k x n
    del barA, barBt
    pa, d = constants.p_prime_accu(N), constants.delta()
    rng = np.random.default_rng(2)
    last = SIZE - 1
    picks = [(0, 0), (0, last), (last, 0), (last, last), (last - 21, 129), (4097, last - 5)]
    picks += [tuple(int(x) for x in rng.integers(SIZE, size=2)) for _ in range(6)]
    for i, j in picks:
        crow = Af[i] @ Bf                  # row i of Cbar
        ccol = Af @ Bf[:, j]               # column j of Cbar
        assert crow.max() < 2.0 ** 53 and ccol.max() < 2.0 ** 53
        ei = scaling.accurate_final_exponent(int(e1A[i]) if nzA[i] else None,
                                             int(crow.max()), pa, d)
        fj = scaling.accurate_final_exponent(int(e1B[j]) if nzB[j] else None,
                                             int(ccol.max()), pa, d)
        c, _, _ = ref.entry(Ah[i], Bh[:, j], ei, fj, N)
        g = float(C_cm[j, i])
        assert np.float64(g).view(np.uint64) == np.float64(c).view(np.uint64), (i, j, g, c)


def test_accurate_every_entry_within_componentwise_bound(accurate_problem):
    A, B, C_cm = accurate_problem
    C = C_cm.t()
    for r0 in range(0, SIZE, 4096):
        Ar = A[r0:r0 + 4096]
        Cn = torch.matmul(Ar, B)
        bound = torch.matmul(Ar.abs(), B.abs()) * 2.0 ** -40
        diff = (C[r0:r0 + 4096] - Cn).abs()
        bad = int((diff > bound).sum())
        assert bad == 0, f"{bad} entries of rows {r0}..{r0 + 4095} outside the bound"
        del Cn, bound, diff
