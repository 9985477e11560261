"""GPU parity of the complex products (ZGEMM, CGEMM) through the C ABI against
the CPU complex oracle: every entry bit for bit at sizes spanning several
GEMM tiles with ragged edges, extreme scalings and edge values, k beyond one
INT32 block, padded leading dimensions, non-finite rows and columns, and
error paths; at 8192^3 sampled entries bit for bit plus a componentwise
bound on every entry."""
import numpy as np
import pytest

from oracle import complex as zref
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

DEV = "cuda:0"
FILL = 7.0 + 7.0j


def _colmajor(M, ld=None):
    """Device buffer holding complex matrix M (r x c) column-major with
    leading dimension ld >= r (a c x ld complex tensor)."""
    r, c = M.shape
    ld = ld or max(1, r)
    buf = np.zeros((c, ld), dtype=M.dtype)
    buf[:, :r] = M.T
    return torch.from_numpy(buf).to(DEV), ld


def _gpu(A, B, N, mode=0, lda=None, ldb=None, ldc=None, single=False):
    ct = np.complex64 if single else np.complex128
    A = np.asarray(A, dtype=ct)
    B = np.asarray(B, dtype=ct)
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = _colmajor(A, lda)
    Bd, ldb = _colmajor(B, ldb)
    ldc = ldc or max(1, m)
    Cd = torch.full((n, ldc), FILL, dtype=torch.complex64 if single else torch.complex128,
                    device=DEV)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    fn = oz.ozaki2_cgemm if single else oz.ozaki2_zgemm
    if mode != 2:
        oz.ensure_workspace(oz.ozaki2_zgemm_workspace_size(m, n, k, N, mode))
    print(f"{fn.__name__} m={m} n={n} k={k} N={N} mode={mode}", flush=True)
    rc = fn(m, n, k, Ad, lda, Bd, ldb, Cd, ldc, N, mode)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    full = Cd.cpu().numpy()
    if ldc > m:
        assert (full[:, m:] == FILL).all(), "padding rows of C were written"
    return full[:, :m].T.copy()


def _same(x, y):
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    w = np.uint64 if x.dtype == np.complex128 else np.uint32
    return x.shape == y.shape and x.dtype == y.dtype and np.array_equal(x.view(w), y.view(w))


@pytest.mark.parametrize("m,n,k,N,mode,phi", [
    (1, 1, 1, 14, 0, 1.0),
    (5, 7, 3, 6, 0, 0.5),
    (33, 65, 100, 14, 0, 2.0),
    (300, 270, 200, 14, 0, 0.5),     # several 256 x 256 tiles, ragged in m, n, k
    (300, 270, 200, 20, 1, 1.0),     # original fast mode, four CRT slices
    (130, 129, 333, 17, 0, 4.0),
    (64, 40, 1000, 9, 1, 2.0),
])
def test_zgemm_matches_oracle(m, n, k, N, mode, phi):
    A, B = inputs.complex_problem(m, n, k, phi, seed=m + n + k + N)
    r = zref.gemm(A, B, N, mode)
    assert _same(_gpu(A, B, N, mode), r["C"])


def test_zgemm_padded_leading_dimensions():
    A, B = inputs.complex_problem(37, 19, 45, 1.0, seed=4)
    r = zref.gemm(A, B, 12)
    assert _same(_gpu(A, B, 12, lda=41, ldb=50, ldc=40), r["C"])


@pytest.mark.parametrize("m,n,k,N,mode", [(70, 90, 150, 7, 0), (33, 300, 64, 5, 1)])
def test_cgemm_matches_oracle(m, n, k, N, mode):
    A, B = inputs.complex_problem(m, n, k, 1.0, seed=k)
    A32, B32 = A.astype(np.complex64), B.astype(np.complex64)
    assert _same(_gpu(A32, B32, N, mode, single=True), zref.cgemm(A32, B32, N, mode))


def test_zgemm_extreme_scaling_and_edge_values():
    """Inputs scaled by 2**+-300 and rows of zeros, powers of two and
    subnormals: still bit for bit."""
    A, B = inputs.complex_problem(40, 30, 70, 2.0, seed=8)
    for c in (2.0 ** 300, 2.0 ** -300):
        r = zref.gemm(A * c, B, 14)
        assert _same(_gpu(A * c, B, 14), r["C"])
    A2 = A.copy()
    A2[3, :] = 0
    A2[5, :] = 2.0 ** -1070 * (1 + 3j)
    A2[7, ::3] = 2.0 ** 40 - 1j * 2.0 ** -30
    B2 = B.copy()
    B2[:, 2] = 0
    B2[::5, 4] = 1j * 2.0 ** -1074
    r = zref.gemm(A2, B2, 16)
    assert _same(_gpu(A2, B2, 16), r["C"])


def test_zgemm_k_beyond_one_int32_block():
    """k > 2^17: the three component GEMMs run over k blocks and accumulate
    modulo p_t; C equals the oracle's, which forms each product over the
    whole k."""
    A, B = inputs.complex_problem(3, 4, 2**17 + 77, 1.0, seed=31)
    r = zref.gemm(A, B, 14)
    assert _same(_gpu(A, B, 14), r["C"])


def test_zgemm_non_finite_rows_and_columns():
    """A NaN or Inf entry makes its row (column) of C NaN in both parts and
    sets the status bit; every other entry is unaffected."""
    A, B = inputs.complex_problem(20, 12, 50, 1.0, seed=2)
    A[4, 7] = complex(np.nan, 0.0)
    B[9, 3] = complex(0.0, np.inf)
    C = _gpu(A, B, 14)
    assert np.isnan(C[4].real).all() and np.isnan(C[4].imag).all()
    assert np.isnan(C[:, 3].real).all() and np.isnan(C[:, 3].imag).all()
    st = oz.ozaki2_get_device_status()
    assert st & 1
    rows = [i for i in range(20) if i != 4]
    cols = [j for j in range(12) if j != 3]
    r = zref.gemm(A[rows], B[:, cols], 14)
    assert _same(C[np.ix_(rows, cols)], r["C"])


def test_zgemm_degenerate_shapes_and_errors():
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    z = lambda cnt: torch.zeros(cnt, dtype=torch.complex128, device=DEV)
    A, B = z(12), z(12)
    C = torch.full((12,), FILL, dtype=torch.complex128, device=DEV)
    # k = 0: C = 0
    assert oz.ozaki2_zgemm(3, 4, 0, A, 3, B, 1, C, 3, 14, 0) == 0
    torch.cuda.synchronize()
    assert (C.cpu().numpy() == 0).all()
    # m = 0 or n = 0: nothing written
    C.fill_(FILL)
    assert oz.ozaki2_zgemm(0, 4, 3, A, 1, B, 3, C, 1, 14, 0) == 0
    assert oz.ozaki2_zgemm(3, 0, 3, A, 3, B, 3, C, 3, 14, 0) == 0
    torch.cuda.synchronize()
    assert (C.cpu().numpy() == FILL).all()
    # accurate mode is not defined for complex products
    assert oz.ozaki2_zgemm(3, 3, 3, A, 3, B, 3, C, 3, 14, 2) == 4
    # misaligned complex pointers (one binary64 into an entry)
    assert oz.ozaki2_zgemm(2, 2, 2, A.data_ptr() + 8, 2, B, 2, C, 2, 14, 0) == -4
    assert oz.ozaki2_zgemm(2, 2, 2, A, 2, B.data_ptr() + 8, 2, C, 2, 14, 0) == -6
    assert oz.ozaki2_zgemm(2, 2, 2, A, 2, B, 2, C.data_ptr() + 8, 2, 14, 0) == -8
    assert oz.ozaki2_cgemm(2, 2, 2, A.data_ptr() + 4, 2, B, 2, C, 2, 14, 0) == -4


def test_torch_convenience_row_major():
    """oz.zgemm on row-major complex128 tensors computes C^T = B^T A^T in
    column-major terms: the same result as the oracle's A B (transposition
    symmetry of the scaling)."""
    A, B = inputs.complex_problem(50, 45, 60, 1.0, seed=6)
    C = oz.zgemm(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), N=13)
    torch.cuda.synchronize()
    assert _same(C.cpu().numpy(), zref.zgemm(A, B, 13))


# --- full size: 8192^3 complex, N = 14 ------------------------------------------

SIZE, N_FULL, PHI_FULL = 8192, 14, 0.5


@pytest.fixture(scope="module")
def full_complex():
    dev = torch.device(DEV)
    A = inputs.complex_matrix_torch(SIZE, SIZE, PHI_FULL, 0, 0, dev)
    B = inputs.complex_matrix_torch(SIZE, SIZE, PHI_FULL, 0, 1, dev)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((SIZE, SIZE), dtype=torch.complex128, device=dev)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    print(f"ozaki2_zgemm {SIZE}^3 N={N_FULL}", flush=True)
    oz.ensure_workspace(oz.ozaki2_zgemm_workspace_size(SIZE, SIZE, SIZE, N_FULL, 0))
    rc = oz.ozaki2_zgemm(SIZE, SIZE, SIZE, A_cm, SIZE, B_cm, SIZE, C_cm, SIZE, N_FULL, 0)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    del A_cm, B_cm
    yield A, B, C_cm
    del A, B, C_cm
    torch.cuda.empty_cache()


def test_full_size_sampled_entries_bit_exact(full_complex):
    A, B, C_cm = full_complex
    last = SIZE - 1
    rng = np.random.default_rng(3)
    picks = [(0, 0), (last, last), (0, last), (last - 100, 255)]
    picks += [tuple(int(x) for x in rng.integers(SIZE, size=2)) for _ in range(4)]
    for i, j in picks:
        row = A[i].cpu().numpy()
        col = B[:, j].cpu().numpy()
        e, f, _, _ = zref.scale_exponents(row[None, :], col[:, None], N_FULL)
        c, _, _ = zref.entry(row, col, e[0], f[0], N_FULL)
        g = complex(C_cm[j, i].item())
        assert _same(np.array([g]), np.array([c])), (i, j, g, c)


def test_full_size_componentwise_bound(full_complex):
    """|C - AB| <= 2**-40 (|Re A||Re B| + |Im A||Im B| + ...) per part, on
    every entry, against torch's native complex product."""
    A, B, C_cm = full_complex
    C = C_cm.t()
    for r0 in range(0, SIZE, 2048):
        Ar = A[r0:r0 + 2048]
        Cn = torch.matmul(Ar, B)
        absA = Ar.real.abs() + Ar.imag.abs()
        absB = B.real.abs() + B.imag.abs()
        bound = torch.matmul(absA, absB) * 2.0 ** -40
        d = C[r0:r0 + 2048] - Cn
        bad = int(((d.real.abs() > bound) | (d.imag.abs() > bound)).sum())
        assert bad == 0, f"{bad} entries of rows {r0}..{r0 + 2047} outside the bound"
        del Cn, bound, d, absA


def test_zgemm_exact_mode_with_huge_rows():
    """Exact mode on complex inputs, rows and columns beyond 1e154 included:
    bit for bit with the oracle (the fallback pass of the complex row kernel
    and of the component view of B)."""
    A, B = inputs.complex_problem(40, 33, 90, 1.0, seed=64)
    A[5] *= 2.0 ** 700
    B[:, 8] *= 2.0 ** 650
    r = zref.gemm(A, B, 16, 3)
    assert _same(_gpu(A, B, 16, mode=3), r["C"])
