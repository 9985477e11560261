"""GPU parity at the benchmark's full size: m = n = k = 16384, N = 14, entries
(rand - 0.5) exp(0.5 randn), seed 0, launched exactly as bench.py launches it
(column-major operands, library stream, caller workspace).

* Sampled entries, including the four corners and the last tile's rows and
  columns, are computed one by one by the CPU oracle from their full row of A
  and column of B (norms, exponents, residues, N dot products, CRT, unscaling)
  and must match bit for bit.
* Every entry must satisfy a property that holds at any size: its distance
  to the native FP64 product is within 2**-40 (|A||B|)_ij (both products are
  far more accurate than that, so a wrong tile, plane or stride anywhere in
  the 2**28 outputs fails it).
"""
import numpy as np
import pytest

from oracle import constants, ozaki2 as ref, scaling
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

SIZE, N, PHI, SEED = 16384, 14, 0.5, 0


@pytest.fixture(scope="module")
def full_problem():
    dev = torch.device("cuda:0")
    A = inputs.ozaki_matrix_torch(SIZE, SIZE, PHI, SEED, 0, dev)   # row-major m x k
    B = inputs.ozaki_matrix_torch(SIZE, SIZE, PHI, SEED, 1, dev)   # row-major k x n
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((SIZE, SIZE), dtype=torch.float64, device=dev)
    ws_bytes = oz.ozaki2_workspace_size(SIZE, SIZE, SIZE, N, 0)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    assert oz.ozaki2_set_workspace(ws_ptr, ws_bytes) == 0
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    rc = oz.ozaki2_dgemm(SIZE, SIZE, SIZE, A_cm, SIZE, B_cm, SIZE, C_cm, SIZE, N, 0)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    assert oz.ozaki2_set_workspace(None, 0) == 0
    del ws, A_cm, B_cm
    yield A, B, C_cm
    del A, B, C_cm
    torch.cuda.empty_cache()


def test_sampled_entries_bit_exact(full_problem):
    A, B, C_cm = full_problem
    rng = np.random.default_rng(1)
    last = SIZE - 1
    picks = [(0, 0), (0, last), (last, 0), (last, last), (last - 37, 255), (256, last - 3)]
    picks += [tuple(int(x) for x in rng.integers(SIZE, size=2)) for _ in range(6)]
    pp = constants.p_prime_prop(N)
    for i, j in picks:
        row = A[i].cpu().numpy()
        col = B[:, j].cpu().numpy()
        ei = scaling.alg2_log2_mu(scaling.norm_sq_ru(row), pp)
        fj = scaling.alg2_log2_mu(scaling.norm_sq_ru(col), pp)
        c, _, _ = ref.entry(row, col, ei, fj, N)
        g = float(C_cm[j, i])
        assert np.float64(g).view(np.uint64) == np.float64(c).view(np.uint64), (i, j, g, c)


def test_every_entry_within_componentwise_bound(full_problem):
    A, B, C_cm = full_problem
    C = C_cm.t()
    # blocks of rows keep the temporaries small
    for r0 in range(0, SIZE, 4096):
        Ar = A[r0:r0 + 4096]
        Cn = torch.matmul(Ar, B)
        bound = torch.matmul(Ar.abs(), B.abs()) * 2.0 ** -40
        diff = (C[r0:r0 + 4096] - Cn).abs()
        bad = int((diff > bound).sum())
        assert bad == 0, f"{bad} entries of rows {r0}..{r0 + 4095} outside the bound"
        del Cn, bound, diff


def test_skinny_full_size_fused_equals_unfused_and_oracle():
    """m = 65536, n = 64, k = 4096 (the skinny configuration), N = 14: the
    fused kernel's C equals the separate kernels' on all 2^22 entries and the
    oracle on sampled entries, bit for bit."""
    dev = torch.device("cuda:0")
    m, n, k, N = 65536, 64, 4096, 14
    A = inputs.ozaki_matrix_torch(m, k, 1.0, 0, 0, dev)
    B = inputs.ozaki_matrix_torch(k, n, 1.0, 0, 1, dev)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    outs = []
    for tile in (0, 3):
        C_cm = torch.empty((n, m), dtype=torch.float64, device=dev)
        assert oz.ozaki2_set_tile(tile) == 0
        print(f"skinny {m}x{n}x{k} tile policy {tile}", flush=True)
        oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, N, 0))
        assert oz.ozaki2_dgemm(m, n, k, A_cm, m, B_cm, k, C_cm, m, N, 0) == 0
        torch.cuda.synchronize()
        outs.append(C_cm)
    oz.ozaki2_set_tile(0)
    assert torch.equal(outs[0].view(torch.int64), outs[1].view(torch.int64))
    pp = constants.p_prime_prop(N)
    rng = np.random.default_rng(5)
    for i, j in [(0, 0), (m - 1, n - 1), (12345, 17)] + [
            tuple(int(x) for x in (rng.integers(m), rng.integers(n))) for _ in range(5)]:
        row, col = A[i].cpu().numpy(), B[:, j].cpu().numpy()
        ei = scaling.alg2_log2_mu(scaling.norm_sq_ru(row), pp)
        fj = scaling.alg2_log2_mu(scaling.norm_sq_ru(col), pp)
        c, _, _ = ref.entry(row, col, ei, fj, N)
        g = float(outs[0][j, i])
        assert np.float64(g).view(np.uint64) == np.float64(c).view(np.uint64), (i, j)
