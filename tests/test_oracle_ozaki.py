"""Pins for the sliced-integer product oracle: exact digit expansions, the
truncation bound against exact rational products, and the complex form."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ozaki


def test_digits_reconstruct_the_rounded_value_exactly():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-0.5, 0.5, 1000), [0.5 - 1e-17, -0.5 + 1e-17, 0.0]])
    for s in (3, 5, 8):
        D = ozaki.digits(x, s)
        assert D[1:].min() >= -64 and D[1:].max() <= 63 and np.abs(D[0]).max() <= 65
        X = np.rint(np.ldexp(x, 7 * s)).astype(np.int64)
        rec = sum(D[i].astype(object) * 128 ** (s - 1 - i) for i in range(s))
        assert all(int(a) == int(b) for a, b in zip(rec, X))


def test_scales_bound_every_entry():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((7, 9)) * 10.0 ** rng.uniform(-5, 5, (7, 1))
    A[3] = 0.0
    e = ozaki.scales(A, 1)
    assert np.all(np.abs(A) < np.ldexp(0.5, e)[:, None])
    assert e[3] == 0


@pytest.mark.parametrize("s", [2, 4, 7, 8])
def test_emulated_product_within_bound_of_exact(s):
    rng = np.random.default_rng(s)
    A = rng.standard_normal((6, 11)) * 10.0 ** rng.uniform(-3, 3, (6, 1))
    B = rng.standard_normal((11, 5)) * 10.0 ** rng.uniform(-3, 3, (1, 5))
    C = ozaki.gemm_real(A, B, s)
    ex = ozaki.exact_product(A, B)
    bnd = ozaki.error_bound(A, B, s)
    err = np.array([[abs(Fraction(float(C[i, j])) - ex[i][j]) for j in range(5)] for i in range(6)], dtype=float)
    # plus the FP64 rounding of the weighted sum (a few ulp of the line scales)
    assert np.all(err <= bnd + 8 * np.ldexp(2.0 ** -53, ozaki.scales(A, 1)[:, None] + ozaki.scales(B, 0)[None, :]))
    if s >= 7:  # FP64 accuracy relative to the row and column scales
        assert np.all(err <= np.ldexp(11 * 2.0 ** -50, ozaki.scales(A, 1)[:, None] + ozaki.scales(B, 0)[None, :]))
    if s == 2:  # and few slices are visibly coarse
        assert err.max() > 1e-6 * np.abs(C).max()


def test_complex_form():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((5, 8)) + 1j * rng.standard_normal((5, 8))
    B = rng.standard_normal((8, 4)) + 1j * rng.standard_normal((8, 4))
    assert np.abs(ozaki.gemm_complex(A, B, 8) - A @ B).max() < 1e-14
