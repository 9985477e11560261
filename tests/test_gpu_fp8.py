"""GPU parity of the FP8 (E4M3) engine variant (mode | OZ2_ENGINE_FP8): the
residue products formed from two E4M3 digits per residue on the FP8 MFMA
engine, against the oracle's FP8 form of Step 3 (oracle.fp8.product) and
its INT8 products, bit for bit; the final C against the oracle and against
the INT8 engine's C, bit for bit."""
import numpy as np
import pytest

from oracle import fp8 as ref_fp8, ozaki2 as ref
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

DEV = "cuda:0"
FP8 = 16          # OZ2_ENGINE_FP8


def _colmajor(M):
    return torch.from_numpy(np.ascontiguousarray(M.T)).to(DEV)


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


def _gemm(A, B, N, mode, fn=None):
    m, k = A.shape
    n = B.shape[1]
    fn = fn or oz.ozaki2_dgemm
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    Ad, Bd = _colmajor(A), _colmajor(B)
    Cd = torch.full((n, m), 7.0, dtype=dt, device=DEV)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, N, mode))
    rc = fn(m, n, k, Ad, m, Bd, k, Cd, m, N, mode)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    return Cd.cpu().numpy().T.copy()


def _product(A, B, N, mode, t):
    m, k = A.shape
    n = B.shape[1]
    Ad, Bd = _colmajor(A), _colmajor(B)
    Ct = torch.zeros(m * n, dtype=torch.int32, device=DEV)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, N, mode))
    rc = oz.ozaki2_debug_stages(m, n, k, Ad, m, Bd, k, N, mode, t,
                                None, None, None, None, None, None, Ct)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy().reshape(n, m).T.astype(np.int64)


CASES = [
    # (m, n, k, phi, N, seed)
    (300, 280, 520, 1.0, 14, 1),     # several 128-tiles each way, ragged; k over one 512 block
    (37, 301, 1100, 2.0, 20, 2),     # N = 20, three binary32 blocks of k
    (129, 130, 64, 4.0, 8, 3),       # one slab of k
    (1, 1, 1, 1.0, 14, 4),
    (5, 3, 2, 0.5, 2, 5),            # N = 2
]


@pytest.mark.parametrize("m,n,k,phi,N,seed", CASES)
def test_fp8_products_and_result(m, n, k, phi, N, seed):
    print(f"fp8 case m={m} n={n} k={k} phi={phi} N={N} seed={seed}", flush=True)
    A, B = inputs.problem(m, n, k, phi, seed)
    r = ref.gemm(A, B, N, ref.REVISED)
    for t in sorted({0, 1, N - 1}):
        got = _product(A, B, N, FP8, t)
        want = ref_fp8.product(r["RA"][t], r["RB"][t])
        assert np.array_equal(want, r["G"][t])
        if t == 0:      # the p = 256 product is exact modulo 2^32 only
            want = (want + 2**31) % 2**32 - 2**31
        assert np.array_equal(got, want), f"FP8 engine product t={t}"
    C8 = _gemm(A, B, N, FP8)
    assert np.array_equal(_bits(C8), _bits(r["C"]))
    assert np.array_equal(_bits(C8), _bits(_gemm(A, B, N, 0)))


@pytest.mark.parametrize("mode", [1, 3])
def test_fp8_other_fast_modes_equal_int8(mode):
    A, B = inputs.problem(200, 150, 700, 2.5, seed=8)
    C8 = _gemm(A, B, 12, mode | FP8)
    assert np.array_equal(_bits(C8), _bits(_gemm(A, B, 12, mode)))
    assert np.array_equal(_bits(C8), _bits(ref.dgemm(A, B, 12, mode)))


def test_fp8_sgemm_equals_int8():
    A, B = inputs.problem(90, 70, 300, 1.0, seed=9)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    C8 = _gemm(A32, B32, 7, FP8, oz.ozaki2_sgemm)
    Ci = _gemm(A32, B32, 7, 0, oz.ozaki2_sgemm)
    assert np.array_equal(C8.view(np.uint32), Ci.view(np.uint32))
    assert np.array_equal(C8.view(np.uint32), ref.sgemm(A, B, 7).view(np.uint32))


def test_fp8_k_beyond_one_int32_block():
    """k > 2^17: two launches, the second adding its products modulo p_t."""
    m, n, k, N = 4, 3, 2**17 + 3000, 14
    A, B = inputs.problem(m, n, k, 1.0, seed=10)
    C8 = _gemm(A, B, N, FP8)
    assert np.array_equal(_bits(C8), _bits(_gemm(A, B, N, 0)))
    assert np.array_equal(_bits(C8), _bits(ref.dgemm(A, B, N)))


def test_fp8_square_4096_equals_int8_and_sampled_oracle():
    """m = n = k = 4096, N = 14, as the bench calls it: every entry identical
    to the INT8 engine's, and sampled entries to the oracle."""
    size, N = 4096, 14
    A = inputs.ozaki_matrix_torch(size, size, 0.5, 0, 0, DEV)
    B = inputs.ozaki_matrix_torch(size, size, 0.5, 0, 1, DEV)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(size, size, size, N, FP8))
    outs = []
    for mode in (FP8, 0):
        C = torch.empty((size, size), dtype=torch.float64, device=DEV)
        assert oz.ozaki2_dgemm(size, size, size, A_cm, size, B_cm, size, C, size, N, mode) == 0
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0].view(torch.int64), outs[1].view(torch.int64))
    from oracle import constants, scaling
    pp = constants.p_prime_prop(N)
    rng = np.random.default_rng(4)
    for _ in range(6):
        i, j = (int(x) for x in rng.integers(size, size=2))
        row, col = A[i].cpu().numpy(), B[:, j].cpu().numpy()
        ei = scaling.alg2_log2_mu(scaling.norm_sq_ru(row), pp)
        fj = scaling.alg2_log2_mu(scaling.norm_sq_ru(col), pp)
        c, _, _ = ref.entry(row, col, ei, fj, N)
        assert _bits(float(outs[0][j, i])) == _bits(c)


def test_fp8_unsupported_combinations():
    A = torch.zeros(16, dtype=torch.float64, device=DEV)
    oz.ensure_workspace(1 << 20)
    # accurate mode, complex products and batches stay on the INT8 engine
    assert oz.ozaki2_dgemm(4, 4, 4, A, 4, A, 4, A, 4, 14, 2 | FP8) == 4
    assert oz.ozaki2_zgemm(2, 2, 2, A, 2, A, 2, A, 2, 14, FP8) == 4
    rc, _, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14)], mode=FP8)
    assert rc == -3
