"""CPU oracle for Ozaki scheme II DGEMM/SGEMM emulation (Kawakami & Takahashi,
"Improved Scaling for Fast Mode of Ozaki Scheme II").

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product library never imports, links or calls it, and it imports nothing
from the product.

The oracle is written to be read against the paper: plain Python integers,
``fractions.Fraction`` for every rounding decision, ``decimal`` for the base-2
logarithm, and numpy only for exact int64 matrix products.  It is slow on
purpose.

Modules
-------
fp         exact rounding of rationals to binary32/binary64 (RN/RU/RD) and the
           correctly rounded binary32 log2 that stands in for the vendor fast log2
constants  Step 1 of Section 2.2 (moduli, P, P_i, q_i) and the single-precision
           constants P'_prop, P'_fast, P'_accu and delta of Sections 2.3 and 4
scaling    the scale exponents: Algorithm 2 (proposed), Algorithm 1 (original
           fast mode) and accurate mode (Section 2.3)
ozaki2     Steps 2-4 of Section 2.2: integers, residues, INT8 products, CRT,
           unscaling
reference  exact rational products and the error metrics used to report accuracy

Where the paper is silent or garbled, the docstring of the function that has
to choose states the reading it takes.
"""
