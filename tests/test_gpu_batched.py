"""GPU: the batched, graph-replayed path gives exactly the results of one
ozaki2_dgemm call per problem, for uneven shapes and per-problem N."""
import numpy as np
import pytest

from oracle import ozaki2 as ref
from paper_2606_29129_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2606_29129_amd import ozaki2 as oz  # noqa: E402

DEV = "cuda:0"


def _problems(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m, n, k = (int(x) for x in np.exp(rng.uniform(np.log(1), np.log(300), 3)).round())
        N = int(rng.choice([6, 8, 14, 17, 20]))
        phi = float(rng.uniform(0.5, 3.0))
        A, B = inputs.problem(m, n, k, phi, seed=1000 * seed + i)
        out.append((A, B, N))
    return out


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("seed", [1, 2])
def test_batched_equals_single_calls_and_oracle(seed):
    probs = _problems(seed, 24)
    pairs = [(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)) for A, B, _ in probs]
    Ns = [N for _, _, N in probs]
    print(f"batch of {len(probs)}: shapes {[a.shape + (b.shape[1],) for a, b, _ in probs][:6]} ...",
          flush=True)
    for rep in range(2):   # the second call replays the cached graph
        outs = oz.dgemm_batched(pairs, Ns)
        torch.cuda.synchronize()
        for (A, B, N), (Ad, Bd), C in zip(probs, pairs, outs):
            single = oz.dgemm(Ad, Bd, N=N).cpu().numpy()
            assert np.array_equal(_bits(C.cpu().numpy()), _bits(single))
    for (A, B, N), C in list(zip(probs, outs))[:6]:
        assert np.array_equal(_bits(C.cpu().numpy()), _bits(ref.dgemm(A, B, N)))


def test_batched_replay_with_new_data_and_edge_problems():
    probs = _problems(3, 8)
    pairs = [(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)) for A, B, _ in probs]
    Ns = [N for _, _, N in probs]
    oz.dgemm_batched(pairs, Ns)
    # same shapes, new values: the graph is replayed with fresh pointers
    pairs2 = [(a * -3.0, b * 0.5) for a, b in pairs]
    outs = oz.dgemm_batched(pairs2, Ns)
    torch.cuda.synchronize()
    for (a, b), N, C in zip(pairs2, Ns, outs):
        assert np.array_equal(_bits(C.cpu().numpy()), _bits(oz.dgemm(a, b, N=N).cpu().numpy()))
    # problems with k = 0 and m = 0 next to a normal one
    A0 = torch.zeros((5, 0), dtype=torch.float64, device=DEV)
    B0 = torch.zeros((0, 4), dtype=torch.float64, device=DEV)
    outs = oz.dgemm_batched([(A0, B0), pairs[0]], [14, Ns[0]])
    torch.cuda.synchronize()
    assert (outs[0].cpu().numpy() == 0.0).all()
    assert np.array_equal(_bits(outs[1].cpu().numpy()),
                          _bits(oz.dgemm(*pairs[0], N=Ns[0]).cpu().numpy()))


def test_batched_autotuned_then_given_N_same_shapes():
    """The same shapes first with N = 0 (the autotuner's phi scratch moves the
    batch's tables further into the workspace) and then with the N it chose:
    the second call is a different plan and must write its own outputs,
    bit-identical to the first call's and to single calls; a batch call
    after single calls (which reuse the workspace) still gives the same
    bits."""
    probs = _problems(5, 10)
    pairs = [(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)) for A, B, _ in probs]
    outs1, Ns = oz.dgemm_batched(pairs, 0, target=1e-15, return_N=True)
    outs2 = oz.dgemm_batched(pairs, Ns)
    torch.cuda.synchronize()
    singles = [oz.dgemm(a, b, N=N).cpu().numpy() for (a, b), N in zip(pairs, Ns)]
    outs3 = oz.dgemm_batched(pairs, Ns)
    torch.cuda.synchronize()
    for c1, c2, c3, s in zip(outs1, outs2, outs3, singles):
        assert np.array_equal(_bits(c1.cpu().numpy()), _bits(s))
        assert np.array_equal(_bits(c2.cpu().numpy()), _bits(s))
        assert np.array_equal(_bits(c3.cpu().numpy()), _bits(s))


def test_batched_large_ragged_problems_equal_single_calls():
    """Problems up to 1500 x 1100 (many tiles per plane, split over XCDs by the
    work ordering) next to small ones, ragged in every dimension: every
    result bit-identical to one ozaki2_dgemm call per problem (which picks
    its own GEMM tile), and sampled entries to the oracle."""
    shapes = [(1024, 768, 300, 14), (512, 512, 1000, 17), (1500, 1100, 200, 20),
              (1000, 1020, 129, 8), (700, 600, 64, 12), (100, 2000, 500, 14),
              (1024, 1024, 1, 6), (37, 45, 1100, 19), (513, 1537, 77, 10)]
    rng = np.random.default_rng(21)
    pairs, Ns = [], []
    for i, (m, n, k, N) in enumerate(shapes):
        A, B = inputs.problem(m, n, k, float(rng.uniform(0.5, 2.5)), seed=300 + i)
        pairs.append((torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)))
        Ns.append(N)
    print(f"shapes {shapes}", flush=True)
    for rep in range(2):
        outs = oz.dgemm_batched(pairs, Ns)
        torch.cuda.synchronize()
        for (a, b), N, C in zip(pairs, Ns, outs):
            assert np.array_equal(_bits(C.cpu().numpy()), _bits(oz.dgemm(a, b, N=N).cpu().numpy()))
    # a few entries of the largest problem against the oracle, entry by entry
    A, B = (x.cpu().numpy() for x in pairs[2])
    C = outs[2].cpu().numpy()
    for r, c in [(0, 0), (1499, 1099), (777, 3), (5, 1024)]:
        want = ref.dgemm(A[r:r + 1], B[:, c:c + 1], Ns[2])
        # one row and one column give the same exponents as in the full
        # problem (they depend only on that row's and column's norms)
        assert np.array_equal(_bits(C[r:r + 1, c:c + 1]), _bits(want))


def test_batched_argument_errors():
    rc, bad, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14),
                                          (4, 4, 4, 1, 2, 1, 4, 1, 4, 14)])
    assert rc == -5 and bad == 1
    rc, _, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14)], mode=2)
    assert rc == -3
    rc, _, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14)], mode=3)
    assert rc == -3


def test_batched_nonfinite_row_sets_status_and_nan_row():
    """A NaN entry in one problem of a batch: that problem's output row is
    NaN, everything else is unchanged, and the device status reports the
    non-finite input once (reading it clears it)."""
    probs = _problems(4, 6)
    pairs = [(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)) for A, B, _ in probs]
    Ns = [N for _, _, N in probs]
    oz.ozaki2_get_device_status()            # clear whatever earlier calls left
    clean = [c.cpu().numpy() for c in oz.dgemm_batched(pairs, Ns)]
    assert oz.ozaki2_get_device_status() == 0
    bad = 2
    Abad = pairs[bad][0].clone()
    Abad[0, 0] = float("nan")
    pairs2 = list(pairs)
    pairs2[bad] = (Abad, pairs[bad][1])
    outs = [c.cpu().numpy() for c in oz.dgemm_batched(pairs2, Ns)]
    assert oz.ozaki2_get_device_status() == 1   # OZ2_STATUS_NONFINITE
    assert oz.ozaki2_get_device_status() == 0
    for i, (C, C0) in enumerate(zip(outs, clean)):
        if i == bad:
            assert np.isnan(C[0]).all()
            assert np.array_equal(_bits(C[1:]), _bits(C0[1:]))
        else:
            assert np.array_equal(_bits(C), _bits(C0))


def _phi_ref(X, vectors):
    """The estimator the library documents, one vector at a time in numpy:
    the rows (or columns) of X, each with its first max(2, 2^20 / count)
    entries; variance of log|x| within each vector pooled over them (zeros
    and non-finite entries skipped, vectors with fewer than two left out)."""
    X = np.asarray(X, np.float64)
    vecs = X if vectors == 0 else X.T
    L = min(vecs.shape[1], max(2, (1 << 20) // max(vecs.shape[0], 1)))
    W = D = 0.0
    for v in vecs[:, :L]:
        x = np.log(np.abs(v[(v != 0) & np.isfinite(v)]))
        if x.size >= 2:
            W += float(((x - x.mean()) ** 2).sum())
            D += x.size - 1
    return float(np.sqrt(max(W / D - 1.0, 0.0))) if D > 0 else 0.0


@pytest.mark.parametrize("rows,cols,ld,phi", [(300, 200, 300, 0.5), (1000, 1500, 1003, 2.7),
                                              (4, 5, 9, 1.0), (2048, 1024, 2048, 4.0),
                                              (20000, 64, 20000, 1.5)])
@pytest.mark.parametrize("vectors", [0, 1])
def test_estimate_phi_matches_numpy(rows, cols, ld, phi, vectors):
    X = inputs.ozaki_matrix(rows, cols, phi, seed=rows)
    if rows > 10:
        X[::7] = 0.0                      # zero rows (and zero entries of columns) skipped
        X[3, 2] = np.inf
    buf = np.zeros((cols, ld))            # column-major with leading dimension ld
    buf[:, :rows] = X.T
    oz.ensure_workspace(1024)              # the estimate's scratch
    dX = torch.from_numpy(buf).to(DEV)
    got = oz.ozaki2_estimate_phi(rows, cols, dX, ld, vectors)
    want = _phi_ref(X, vectors)
    assert abs(got - want) <= 1e-9 * max(1.0, want)
    if rows * cols > 5000:
        assert abs(got - phi) < 0.1      # and it estimates the distribution's phi
    # rows (columns) scaled by their own powers of two: the same estimate
    rng = np.random.default_rng(rows + vectors)
    if vectors == 0:
        Y = X * np.ldexp(1.0, rng.integers(-200, 200, rows))[:, None]
    else:
        Y = X * np.ldexp(1.0, rng.integers(-200, 200, cols))[None, :]
    buf[:, :rows] = Y.T
    got2 = oz.ozaki2_estimate_phi(rows, cols, torch.from_numpy(buf).to(DEV), ld, vectors)
    assert abs(got2 - got) <= 1e-9 * max(1.0, got)


def test_batched_autotune_picks_the_python_N_and_same_bits():
    """N = 0 in a batch: the library's N_used equals the Python autotuner's
    pick for the same estimates, and C is bit-identical to the batch with
    those N given explicitly and to single calls."""
    from paper_2606_29129_amd import autotune
    rng = np.random.default_rng(9)
    pairs, want = [], []
    for i in range(12):
        m, n, k = (int(x) for x in np.exp(rng.uniform(np.log(8), np.log(400), 3)).round())
        phi = float(rng.uniform(0.5, 3.0))
        A, B = inputs.problem(m, n, k, phi, seed=500 + i)
        pairs.append((torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)))
        ph = max(_phi_ref(A, 0), _phi_ref(B, 1))      # the rows of A, the columns of B
        want.append(autotune.pick_N(k, ph, 1e-15))
    outs, used = oz.dgemm_batched(pairs, 0, target=1e-15, return_N=True)
    assert used == want
    explicit = oz.dgemm_batched(pairs, used)
    torch.cuda.synchronize()
    for (a, b), N, C, E in zip(pairs, used, outs, explicit):
        assert np.array_equal(_bits(C.cpu().numpy()), _bits(E.cpu().numpy()))
        assert np.array_equal(_bits(C.cpu().numpy()), _bits(oz.dgemm(a, b, N=N).cpu().numpy()))
    # mixed: some N given, some left to the library; degenerate problems report 0
    e = torch.zeros((0, 5), dtype=torch.float64, device=DEV)
    f = torch.zeros((5, 3), dtype=torch.float64, device=DEV)
    _, used2 = oz.dgemm_batched(pairs[:3] + [(e, f)], [7, 0, 0, 0], target=1e-15, return_N=True)
    assert used2 == [7, want[1], want[2], 0]


def test_batched_original_fast_mode_equals_single_calls_and_oracle():
    """Mode 1 (Algorithm 1, Section 2.3) through the batched path -- its own
    route through the row and column maxima and the Algorithm 1 fold --
    on uneven shapes: every problem bit-identical to one ozaki2_dgemm call
    in mode 1, and the small problems to the oracle."""
    probs = _problems(6, 14)
    pairs = [(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)) for A, B, _ in probs]
    Ns = [N for _, _, N in probs]
    print(f"original mode batch: shapes {[a.shape + (b.shape[1],) for a, b, _ in probs][:6]} ...",
          flush=True)
    for rep in range(2):   # the second call replays the graph
        outs = oz.dgemm_batched(pairs, Ns, mode="original")
        torch.cuda.synchronize()
        for (Ad, Bd), N, C in zip(pairs, Ns, outs):
            single = oz.dgemm(Ad, Bd, N=N, mode="original").cpu().numpy()
            assert np.array_equal(_bits(C.cpu().numpy()), _bits(single))
    for (A, B, N), C in list(zip(probs, outs))[:5]:
        assert np.array_equal(_bits(C.cpu().numpy()), _bits(ref.dgemm(A, B, N, ref.ORIGINAL)))
    # the two modes differ on these inputs (Algorithm 1 is not Algorithm 2)
    rev = oz.dgemm_batched(pairs, Ns)
    torch.cuda.synchronize()
    assert any(not np.array_equal(_bits(a.cpu().numpy()), _bits(b.cpu().numpy()))
               for a, b in zip(rev, outs))
