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


def test_batched_argument_errors():
    rc, bad = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14), (4, 4, 4, 1, 2, 1, 4, 1, 4, 14)])
    assert rc == -5 and bad == 1
    rc, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14)], mode=2)
    assert rc == -3
    rc, _ = oz.ozaki2_dgemm_batched([(4, 4, 4, 1, 4, 1, 4, 1, 4, 14)], mode=3)
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
