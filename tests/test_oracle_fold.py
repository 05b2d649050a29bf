"""Pins of the float map-reduce oracle (Section 4.2) against exact arithmetic and closed forms."""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

from oracle import fold

U = 2.0 ** -53  # unit roundoff of binary64


def test_alternating_harmonic_small_n_exact():
    # exact rational sum; the oracle rounds each term and then the sum once
    for n in list(range(0, 40)) + [99, 200]:
        exact = sum((Fraction(1, i) if i % 2 else -Fraction(1, i)) for i in range(1, n + 1))
        got = fold.fold_sum(fold.ALT_HARMONIC, n)
        bound = U * (fold.abs_sum(fold.ALT_HARMONIC, n) + abs(float(exact)))
        assert abs(Fraction(got) - exact) <= Fraction(bound), n


def test_sqrt_small_n_exact():
    getcontext().prec = 50
    for n in list(range(0, 40)) + [99, 200]:
        exact = sum((Decimal(i).sqrt() for i in range(1, n + 1)), Decimal(0))
        got = fold.fold_sum(fold.SQRT, n)
        bound = U * (fold.abs_sum(fold.SQRT, n) + float(exact))
        assert abs(Decimal(got) - exact) <= Decimal(bound), n


@pytest.mark.parametrize("n", [10 ** 6, 10 ** 6 + 1, 1_234_567])
def test_alternating_harmonic_limit_ln2(n):
    # S_n = ln 2 + (-1)^(n+1) (1/(2n) - 1/(4n^2) + O(n^-4)): the limit the paper quotes, with
    # the tail of the alternating series (its Euler transform)
    s = fold.fold_sum(fold.ALT_HARMONIC, n)
    approx = math.log(2) + (-1) ** (n + 1) * (1 / (2 * n) - 1 / (4 * n * n))
    assert abs(s - approx) <= 4e-15 + 1 / n ** 3
    # the partial sums alternate around ln 2
    assert (s > math.log(2)) == (n % 2 == 1)


@pytest.mark.parametrize("n", [10 ** 6, 10 ** 6 + 1, 1_234_567])
def test_sqrt_sum_euler_maclaurin(n):
    # sum_{i<=n} sqrt(i) = 2/3 n^(3/2) + 1/2 n^(1/2) + zeta(-1/2) + 1/24 n^(-1/2)
    #                      - 1/1920 n^(-5/2) + O(n^(-9/2))
    getcontext().prec = 50
    zeta = Decimal("-0.20788622497735456601730672539704930222626853128767")
    N = Decimal(n)
    r = N.sqrt()
    em = Decimal(2) / 3 * N * r + r / 2 + zeta + 1 / (24 * r) - 1 / (1920 * N * N * r)
    s = fold.fold_sum(fold.SQRT, n)
    assert abs(Decimal(s) - em) <= Decimal(2 * math.ulp(s))


def test_last_term_and_empty():
    assert fold.fold_sum(fold.SQRT, 0) == 0.0 and fold.fold_sum(fold.ALT_HARMONIC, 0) == 0.0
    assert fold.fold_sum(fold.SQRT, 1) == 1.0 and fold.fold_sum(fold.ALT_HARMONIC, 1) == 1.0
    assert fold.fold_sum(fold.ALT_HARMONIC, 2) == 0.5
    for kind in (fold.SQRT, fold.ALT_HARMONIC):
        for n in (2, 17, 1000, 4097):
            d = fold.fold_sum(kind, n) - fold.fold_sum(kind, n - 1)
            t = float(fold.terms(kind, n, n + 1)[0])
            tol = 2 * U * (abs(fold.fold_sum(kind, n)) + abs(fold.fold_sum(kind, n - 1)))
            assert abs(d - t) <= tol + U * abs(t), (kind, n)
