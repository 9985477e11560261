"""Host-side logic of the N autotuner (CPU only)."""
import ctypes
import json
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2606_29129_amd import autotune, inputs


@pytest.mark.parametrize("phi", [0.5, 1.0, 2.0, 3.0])
def test_estimate_phi_recovers_the_generator_spread(phi):
    A = inputs.ozaki_matrix(200, 2000, phi, seed=5)
    assert abs(autotune.estimate_phi(A, "rows") - phi) < 0.08 * max(1.0, phi)
    assert abs(autotune.estimate_phi(A, "cols") - phi) < 0.08 * max(1.0, phi)


def _pooled_phi(vectors):
    """The estimator's definition, one vector at a time."""
    W = D = 0.0
    for v in vectors:
        v = np.asarray(v, np.float64)
        x = np.log(np.abs(v[(v != 0) & np.isfinite(v)]))
        if x.size >= 2:
            W += float(((x - x.mean()) ** 2).sum())
            D += x.size - 1
    return math.sqrt(max(W / D - 1.0, 0.0)) if D > 0 else 0.0


def test_estimate_phi_is_the_pooled_within_vector_spread_and_ignores_vector_scales():
    """Against the definition written out vector by vector (with zeros,
    infinities and a vector of one entry), on both orientations and the
    sample sizes of the rule; scaling each row (column) by its own power of
    two leaves it unchanged, while the variance of all entries taken
    together grows."""
    rng = np.random.default_rng(11)
    X = inputs.ozaki_matrix(300, 40, 1.5, seed=2)
    X[5, :] = 0.0
    X[7, 3] = np.inf
    X[9, 1:] = 0.0
    assert abs(autotune.estimate_phi(X, "rows") - _pooled_phi(X)) < 1e-12
    assert abs(autotune.estimate_phi(X, "cols") - _pooled_phi(X.T)) < 1e-12
    big = inputs.ozaki_matrix(4096, 600, 0.7, seed=3)       # rows keep 256 entries each
    assert abs(autotune.estimate_phi(big, "rows") - _pooled_phi(big[:, :256])) < 1e-12
    assert abs(autotune.estimate_phi(big.T, "cols") - _pooled_phi(big[:, :256])) < 1e-12
    wide = inputs.ozaki_matrix(400, 5000, 0.7, seed=4)      # columns keep 209 entries each
    assert abs(autotune.estimate_phi(wide, "cols") - _pooled_phi(wide[:209, :].T)) < 1e-12
    rs = np.ldexp(1.0, rng.integers(-300, 300, X.shape[0]))[:, None]
    cs = np.ldexp(1.0, rng.integers(-300, 300, X.shape[1]))[None, :]
    assert abs(autotune.estimate_phi(X * rs, "rows") - autotune.estimate_phi(X, "rows")) < 1e-9
    assert abs(autotune.estimate_phi(X * cs, "cols") - autotune.estimate_phi(X, "cols")) < 1e-9
    flat = np.log(np.abs((X * rs)[(X != 0) & np.isfinite(X)]))
    assert math.sqrt(max(flat.var() - 1.0, 0.0)) > 10 * autotune.estimate_phi(X, "rows")


def test_exact_dot_and_rel_err():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = rng.standard_normal(40) * np.exp(3 * rng.standard_normal(40))
        b = rng.standard_normal(40) * np.exp(3 * rng.standard_normal(40))
        n, e = autotune.exact_dot(a, b)
        exact = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))
        assert Fraction(n) * (Fraction(2) ** e) == exact
        c = float(exact)
        assert autotune.rel_err(c, (n, e)) <= 2.0 ** -53
    assert autotune.exact_dot([0.0, 1.0], [5.0, 0.0]) == (0, 0)
    assert autotune.rel_err(0.0, (0, 0)) == 0.0


def test_pick_N_is_monotone_in_target_k_and_phi():
    # synthetic table: error halves with each modulus, grows with k and phi
    tab = {"errors": {}}
    for k in autotune.K_GRID:
        tab["errors"][str(k)] = {}
        for phi in autotune.PHI_GRID:
            tab["errors"][str(k)][str(phi)] = {
                str(N): 2.0 ** (-4 * N) * k * math.exp(2 * phi) for N in autotune.N_GRID}
    Ns = [autotune.pick_N(512, 1.2, t, tab) for t in (1e-8, 1e-12, 1e-15, 1e-18)]
    assert Ns == sorted(Ns)
    assert autotune.pick_N(64, 0.5, 1e-15, tab) <= autotune.pick_N(2048, 0.5, 1e-15, tab)
    assert autotune.pick_N(256, 0.5, 1e-15, tab) <= autotune.pick_N(256, 3.0, 1e-15, tab)
    # beyond the grid and unreachable targets
    assert autotune.pick_N(10**6, 9.0, 1e-300, tab) == 20


def test_library_tile_choice_matches_measurements():
    """The library's automatic tile (ozaki2_get_tile, host logic) is within
    2% of the fastest forced tile on every measured shape, and the committed
    fit reproduces the library's constants."""
    from paper_2606_29129_amd import ozaki2 as oz
    with open(autotune.TILE_TABLE) as f:
        table = json.load(f)
    for rec in table["shapes"]:
        for N in table["Ns"]:
            ms = {t: rec["ms"][f"{N}/{t}"] for t in autotune.TILES}
            pick = oz.ozaki2_get_tile(rec["m"], rec["n"], rec["k"], N)
            assert ms[pick] <= 1.02 * min(ms.values()), (rec["m"], rec["n"], rec["k"], N, pick)
    rate, fixed, tot, worst = autotune.fit_tile_model(table)
    assert rate == {1: 1.0, 2: 0.75, 3: 0.45} and fixed == {1: 2, 2: 0, 3: 0}
    assert worst < 0.01


def test_library_pick_equals_python_pick():
    """ozaki2_autotune_N (host code in the library, over the generated table
    header) picks what autotune.pick_N picks from the JSON, on and between
    the grid points, beyond both ends, for targets 1e-6 .. 1e-17."""
    import itertools
    from paper_2606_29129_amd import ozaki2 as oz
    ks = [1, 64, 65, 200, 256, 1000, 2048, 2049, 8192, 10000, 16384, 20000, 2**20]
    phis = [0.0, 0.3, 0.5, 0.5000000001, 0.7, 1.0, 1.25, 2.0, 2.9, 3.0, 3.5, 4.0, 6.0]
    targets = [1e-6, 1e-9, 1e-12, 1e-13, 3e-14, 1e-15, 4e-16, 1e-16, 1e-17]
    for k, phi, tg in itertools.product(ks, phis, targets):
        assert oz.ozaki2_autotune_N(k, phi, tg) == autotune.pick_N(k, phi, tg), (k, phi, tg)


def test_table_header_is_generated_from_the_json():
    with open(autotune.HEADER) as f:
        assert f.read() == autotune.header_text()


def test_autotune_argument_errors():
    from paper_2606_29129_amd import ozaki2 as oz
    lib = oz.lib()
    N = ctypes.c_int(0)
    assert lib.ozaki2_autotune_N(-1, 1.0, 1e-15, ctypes.byref(N)) == -1
    assert lib.ozaki2_autotune_N(10, -1.0, 1e-15, ctypes.byref(N)) == -2
    assert lib.ozaki2_autotune_N(10, float("nan"), 1e-15, ctypes.byref(N)) == -2
    assert lib.ozaki2_autotune_N(10, 1.0, 0.0, ctypes.byref(N)) == -3
    assert lib.ozaki2_autotune_N(10, 1.0, 1e-15, None) == -4
    phi = ctypes.c_double(0)
    assert lib.ozaki2_estimate_phi(-1, 1, None, 1, 0, ctypes.byref(phi)) == -1
    assert lib.ozaki2_estimate_phi(4, -1, None, 4, 0, ctypes.byref(phi)) == -2
    assert lib.ozaki2_estimate_phi(4, 4, None, 4, 0, ctypes.byref(phi)) == -3
    assert lib.ozaki2_estimate_phi(4, 4, 8, 3, 0, ctypes.byref(phi)) == -4
    assert lib.ozaki2_estimate_phi(4, 4, 8, 4, 2, ctypes.byref(phi)) == -5
    assert lib.ozaki2_estimate_phi(4, 4, 8, 4, 1, None) == -6
    assert lib.ozaki2_estimate_phi(0, 4, None, 1, 1, ctypes.byref(phi)) == 0 and phi.value == 0.0
    # a batch with N = 0 needs a target; nothing is launched
    prob = oz.Oz2Problem(4, 4, 4, 8, 4, 8, 4, 8, 4, 0, 0)
    arr = (oz.Oz2Problem * 1)(prob)
    bad = ctypes.c_int(0)
    assert lib.ozaki2_dgemm_batched(1, arr, 0, 0.0, ctypes.byref(bad)) == -4
    assert lib.ozaki2_dgemm_batched(1, arr, 0, 2.0, ctypes.byref(bad)) == -4


def test_pick_N_on_the_committed_table_is_monotone():
    """On the committed calibration: the pick never falls when k or phi grow
    or the target tightens (the envelope), on and between grid points; phi
    beyond the calibrated range gives N = 20; k beyond it never picks fewer
    moduli than at the largest calibrated k."""
    ks = [64, 100, 256, 700, 1024, 2048, 5000, 8192, 16384, 2**16, 2**22]
    phis = [0.0, 0.5, 0.8, 1.0, 1.5, 2.0, 2.2, 2.5, 3.0, 3.7, 4.0]
    targets = [1e-9, 1e-12, 1e-14, 1e-15, 3e-16, 1e-16]
    for t in targets:
        for phi in phis:
            picks = [autotune.pick_N(k, phi, t) for k in ks]
            assert picks == sorted(picks), (phi, t, picks)
        for k in ks:
            picks = [autotune.pick_N(k, phi, t) for phi in phis]
            assert picks == sorted(picks), (k, t, picks)
    for k in ks:
        for phi in phis:
            picks = [autotune.pick_N(k, phi, t) for t in targets]
            assert picks == sorted(picks), (k, phi, picks)
    assert autotune.pick_N(1024, 4.5, 1e-6) == 20
    assert autotune.pick_N(2**22, 0.5, 1e-15) >= autotune.pick_N(16384, 0.5, 1e-15)


def test_error_estimate_is_an_envelope_of_the_table():
    """The estimate at a grid point bounds every tabulated error at or below
    it (k, phi) for the same or a larger N, and grows by sqrt(k/16384)
    beyond the calibrated k."""
    t = autotune.load_table()
    ks = sorted(int(x) for x in t["errors"])
    phis = sorted(float(x) for x in t["errors"][str(ks[0])])
    for k in ks:
        for phi in phis:
            for N in autotune.N_GRID:
                e = autotune.error_estimate(k, phi, N)
                for k2 in ks:
                    for p2 in phis:
                        if k2 <= k and p2 <= phi:
                            for N2 in autotune.N_GRID:
                                if N2 >= N:
                                    assert t["errors"][str(k2)][str(p2)][str(N2)] <= e
    e16 = autotune.error_estimate(16384, 1.0, 14)
    assert autotune.error_estimate(4 * 16384, 1.0, 14) == 2 * e16
    assert autotune.error_estimate(100, 4.01, 14) is None
