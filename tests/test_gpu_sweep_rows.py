"""GPU: the configurations of the measurement sweeps (square throughput,
rectangular and skinny shapes in the three modes, the accuracy sweep's
DGEMM and SGEMM) called as the sweeps call them -- column-major operands
from the device generator, a caller workspace, the library stream -- with
sampled entries of every result computed from scratch by the oracle (the
row's and column's squared norms and exponents, Steps 2-4 for the one
entry) and compared bit for bit.  Each row of the published sweep tables
is one of these calls, so its numbers describe results the oracle
reproduces."""
import numpy as np
import pytest

from oracle import constants, fp, ozaki2 as ref, scaling
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

DEV = "cuda:0"
SAMPLES = 3


def _exponent(v, N, mode):
    if mode == 0:
        return scaling.alg2_log2_mu(scaling.norm_sq_ru(v), constants.p_prime_prop(N))
    if mode == 1:
        return scaling.alg1_log2_mu(scaling.norm_sq_ru(v), float(np.max(np.abs(v))),
                                    constants.p_prime_fast(N), constants.delta())
    if mode == 3:
        return scaling.exact_mode_log2_mu(v, constants.step1(N)[1])[0]
    raise ValueError(mode)


def _accurate_exponents(Ah, Bh, N, picks):
    """Accurate mode (Section 2.3): the oracle's bar matrices over all of A
    and B, the needed rows and columns of their product (exact in binary64:
    integers below 2^53), the oracle's last exponent step."""
    e1A, nzA, barA = scaling.accurate_bars(Ah)
    e1B, nzB, barBt = scaling.accurate_bars(Bh.T)
    Af = barA.astype(np.float64)
    Bf = np.ascontiguousarray(barBt.T.astype(np.float64))
    pa, d = constants.p_prime_accu(N), constants.delta()
    out = []
    for i, j in picks:
        ei = scaling.accurate_final_exponent(int(e1A[i]) if nzA[i] else None,
                                             int((Af[i] @ Bf).max()), pa, d)
        fj = scaling.accurate_final_exponent(int(e1B[j]) if nzB[j] else None,
                                             int((Af @ Bf[:, j]).max()), pa, d)
        out.append((ei, fj))
    return out


def _run_and_check(m, n, k, phi, N, mode, single=False, seed=0):
    print(f"sweep row m={m} n={n} k={k} phi={phi} N={N} mode={mode} single={single}", flush=True)
    A = inputs.ozaki_matrix_torch(m, k, phi, seed, 0, DEV)
    B = inputs.ozaki_matrix_torch(k, n, phi, seed, 1, DEV)
    if single:
        A, B = A.float(), B.float()
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((n, m), dtype=A.dtype, device=DEV)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, N, mode))
    fn = oz.ozaki2_sgemm if single else oz.ozaki2_dgemm
    rc = fn(m, n, k, A_cm, m, B_cm, k, C_cm, m, N, mode)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    del A_cm, B_cm
    rng = np.random.default_rng(1000 + N + 7 * mode)
    picks = [(int(rng.integers(m)), int(rng.integers(n))) for _ in range(SAMPLES)]
    picks[0] = (m - 1, n - 1)       # the last row and column (the tiles' ragged edge)
    if mode == 2:
        exps = _accurate_exponents(A.double().cpu().numpy(), B.double().cpu().numpy(), N, picks)
    fmt = fp.BINARY32 if single else fp.BINARY64
    for s, (i, j) in enumerate(picks):
        row = A[i].double().cpu().numpy()
        col = B[:, j].double().cpu().numpy()
        ei, fj = exps[s] if mode == 2 else (_exponent(row, N, mode), _exponent(col, N, mode))
        want, _, _ = ref.entry(row, col, ei, fj, N, fmt)
        got = C_cm[j, i].item()
        if single:
            assert np.float32(got).view(np.uint32) == np.float32(want).view(np.uint32), (i, j)
        else:
            assert np.float64(got).view(np.uint64) == np.float64(want).view(np.uint64), (i, j)
    del A, B, C_cm
    torch.cuda.empty_cache()


@pytest.mark.parametrize("S", [1024, 4096, 16384])
@pytest.mark.parametrize("phi", [0.5, 4.0])
@pytest.mark.parametrize("N", [12, 20])
def test_throughput_rows(S, phi, N):
    _run_and_check(S, S, S, phi, N, 0)


@pytest.mark.parametrize("m,n,k", [(8192, 8192, 1024), (8192, 8192, 8192),
                                   (8192, 8192, 65536), (65536, 64, 4096)])
@pytest.mark.parametrize("mode", [0, 1])
def test_shapes_rows(m, n, k, mode):
    _run_and_check(m, n, k, 1.0, 14, mode)


def test_shapes_row_accurate_mode():
    _run_and_check(8192, 8192, 1024, 1.0, 14, 2)


@pytest.mark.parametrize("N", [8, 14, 20])
def test_accuracy_rows_dgemm(N):
    _run_and_check(8192, 8192, 8192, 2.0, N, 0)


@pytest.mark.parametrize("N", [5, 9])
def test_accuracy_rows_sgemm(N):
    _run_and_check(8192, 8192, 8192, 2.0, N, 0, single=True)


def test_exact_mode_row():
    _run_and_check(4096, 4096, 4096, 1.0, 14, 3)
