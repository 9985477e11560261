"""Host-side logic of the N autotuner (CPU only)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2606_29129_amd import autotune, inputs


@pytest.mark.parametrize("phi", [0.5, 1.0, 2.0, 3.0])
def test_estimate_phi_recovers_the_generator_spread(phi):
    A = inputs.ozaki_matrix(200, 2000, phi, seed=5)
    assert abs(autotune.estimate_phi(A) - phi) < 0.08 * max(1.0, phi)


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
