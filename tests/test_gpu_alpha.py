"""GPU: the scale experiment of Sections 3.2 and 4 (A = 2^s Ahat, B = 2^s
Bhat for fixed random Ahat, Bhat) at m = n = k = 1024, phi = 0.5, N = 20.

Revised mode (Algorithm 2): the row and column exponents shift by exactly -s
(or, where the binary32 rounding of w lowers one, by -s - 1), and every entry
whose row and column both shifted exactly equals 4^s times the s = 0 result
bit for bit -- the scale invariance the revised scaling is built for.
Original mode (Algorithm 1): its exponents do not follow s; at both ends of
the range the GPU's results equal the oracle's bit for bit (including where
the CRT recovery breaks down).  Sampled entries are recomputed from scratch
by the oracle in both modes."""
import numpy as np
import pytest

from oracle import constants, ozaki2 as ref, scaling
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

DEV = "cuda:0"
S, PHI, N = 1024, 0.5, 20


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


@pytest.fixture(scope="module")
def hat():
    A = inputs.ozaki_matrix_torch(S, S, PHI, 0, 0, DEV)
    B = inputs.ozaki_matrix_torch(S, S, PHI, 0, 1, DEV)
    return A, B


def _run(A, B, mode):
    """C (row-major, on the device) and the row/column exponents."""
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((S, S), dtype=torch.float64, device=DEV)
    eA = torch.zeros(S, dtype=torch.int32, device=DEV)
    eB = torch.zeros(S, dtype=torch.int32, device=DEV)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(S, S, S, N, mode))
    rc = oz.ozaki2_dgemm(S, S, S, A_cm, S, B_cm, S, C_cm, S, N, mode)
    assert rc == 0, oz.ozaki2_status_string(rc)
    rc = oz.ozaki2_debug_stages(S, S, S, A_cm, S, B_cm, S, N, mode, 0, eA, eB)
    assert rc == 0, oz.ozaki2_status_string(rc)
    torch.cuda.synchronize()
    return C_cm.t(), eA.cpu().numpy(), eB.cpu().numpy()


def _oracle_entry(row, col, mode):
    if mode == 0:
        pp = constants.p_prime_prop(N)
        e = scaling.alg2_log2_mu(scaling.norm_sq_ru(row), pp)
        f = scaling.alg2_log2_mu(scaling.norm_sq_ru(col), pp)
    else:
        pf, d = constants.p_prime_fast(N), constants.delta()
        e = scaling.alg1_log2_mu(scaling.norm_sq_ru(row), float(np.max(np.abs(row))), pf, d)
        f = scaling.alg1_log2_mu(scaling.norm_sq_ru(col), float(np.max(np.abs(col))), pf, d)
    return ref.entry(row, col, e, f, N)[0], e, f


def _check_samples(A, B, C, eA, eB, mode, seed):
    rng = np.random.default_rng(seed)
    for _ in range(3):
        i, j = (int(x) for x in rng.integers(S, size=2))
        row, col = A[i].cpu().numpy(), B[:, j].cpu().numpy()
        want, e, f = _oracle_entry(row, col, mode)
        assert (int(eA[i]), int(eB[j])) == (e, f), (i, j)
        assert _bits(float(C[i, j])) == _bits(want), (i, j)


@pytest.mark.parametrize("s", [-10, -5, -1, 3, 10])
def test_revised_scale_invariance(hat, s):
    print(f"alpha revised s={s}", flush=True)
    Ah, Bh = hat
    C0, eA0, eB0 = _run(Ah, Bh, 0)
    a = 2.0 ** s
    A, B = Ah * a, Bh * a
    C1, eA1, eB1 = _run(A, B, 0)
    dA, dB = eA1 - (eA0 - s), eB1 - (eB0 - s)
    assert set(np.unique(dA)) <= {0, -1} and set(np.unique(dB)) <= {0, -1}
    rows = torch.as_tensor(np.nonzero(dA == 0)[0], device=DEV)
    cols = torch.as_tensor(np.nonzero(dB == 0)[0], device=DEV)
    assert rows.numel() >= S - 8 and cols.numel() >= S - 8
    got = C1.index_select(0, rows).index_select(1, cols)
    want = C0.index_select(0, rows).index_select(1, cols) * (a * a)
    assert torch.equal(got.contiguous().view(torch.int64), want.contiguous().view(torch.int64))
    _check_samples(A, B, C1, eA1, eB1, 0, seed=100 + s)


@pytest.mark.parametrize("s", [-10, -2, 10])
def test_original_mode_against_oracle(hat, s):
    print(f"alpha original s={s}", flush=True)
    Ah, Bh = hat
    a = 2.0 ** s
    A, B = Ah * a, Bh * a
    C, eA, eB = _run(A, B, 1)
    _check_samples(A, B, C, eA, eB, 1, seed=200 + s)
