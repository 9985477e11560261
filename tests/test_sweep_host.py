"""The double-double reference of the measurement sweeps against exact
rational dot products (CPU)."""
from fractions import Fraction

import numpy as np

from paper_2606_29129_amd import inputs, sweep


def _exact(a, b):
    return sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))


def test_dd_block_matches_exact_products():
    A = inputs.ozaki_matrix(6, 300, 2.0, 3, 0)
    B = inputs.ozaki_matrix(300, 5, 2.0, 3, 1)
    hi, lo = sweep.dd_block(A, B)
    for i in range(6):
        for j in range(5):
            ex = _exact(A[i], B[:, j])
            got = Fraction(float(hi[i, j])) + Fraction(float(lo[i, j]))
            assert abs(got - ex) <= abs(ex) * Fraction(1, 2 ** 95)


def test_dd_block_cancellation_and_errors():
    # exact cancellation: (x, -x) pairs give 0; errors() counts C != 0 there
    A = np.array([[1e10, 1.0, -1e10]])
    B = np.array([[3.0], [2.0 ** -60], [3.0]])
    hi, lo = sweep.dd_block(A, B)
    assert hi[0, 0] + lo[0, 0] == 2.0 ** -60
    e = sweep.errors(np.array([[2.0 ** -60 * (1 + 2.0 ** -52)]]), (hi, lo), np.abs(A) @ np.abs(B))
    assert e["max_rel"] == 2.0 ** -52
    z = sweep.errors(np.array([[1.0]]), (np.zeros((1, 1)), np.zeros((1, 1))), np.ones((1, 1)))
    assert z["zero_ref_nonzero"] == 1 and z["max_cw"] == 1.0
