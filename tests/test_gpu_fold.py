"""Parity of the float map-reduce kernel (Section 4.2) with the oracle, within the bound the
kernel's addition tree gives: |gpu - oracle| <= (m + 23) u sum|term| + u |sum|, u = 2^-53,
m = the per-thread run length of the kernel's layout."""
import math

import pytest
import torch

from oracle import fold as ofold
from paper_2206_05269_amd import wc

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
KINDS = [wc.WC_FOLD_SQRT, wc.WC_FOLD_ALT_HARMONIC]


def run_length(n):
    g = min(2048, max(1, (n + 255) // 256))
    return (n + 256 * g - 1) // (256 * g)


def bound(kind, n, ref):
    return (run_length(n) + 23) * U * ofold.abs_sum(kind, n) + U * abs(ref)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 12_345, 65_539,
                               524_288, 524_289, 2_000_003])
def test_fold_matches_oracle(kind, n):
    got = wc.fold_sum(kind, n)
    ref = ofold.fold_sum(kind, n)
    assert abs(got - ref) <= bound(kind, n, ref), (got, ref)
    if n <= 1:
        assert got == ref  # nothing to round


@pytest.mark.parametrize("kind", KINDS)
def test_fold_is_deterministic(kind):
    f = wc.FoldSum(kind, 10_000_019)
    a = f.run(10_000_019).clone()
    b = f.run(10_000_019).clone()
    torch.cuda.synchronize()
    assert a.item() == b.item()
    # a smaller call after a larger one on the same workspace
    small = f.run(1000).item()
    assert abs(small - ofold.fold_sum(kind, 1000)) <= bound(kind, 1000, small)


def test_fold_at_the_paper_largest_n():
    # n = 10^8, the largest n of the paper's tables: closed forms at that size
    n = 10 ** 8
    m = run_length(n)
    s = wc.fold_sum(wc.WC_FOLD_ALT_HARMONIC, n)
    h = math.log(n) + 0.5772156649015329 + 1 / (2 * n)  # sum of |term|
    tail = (-1) ** (n + 1) * (1 / (2 * n) - 1 / (4 * n * n))
    assert abs(s - (math.log(2) + tail)) <= (m + 23) * U * h + 1e-14 + 1 / n ** 3
    r = wc.fold_sum(wc.WC_FOLD_SQRT, n)
    zeta = -0.20788622497735456601730672539704930222626853128767
    em = 2 / 3 * n ** 1.5 + 0.5 * n ** 0.5 + zeta + 1 / (24 * n ** 0.5)
    assert abs(r - em) <= (m + 23) * U * r + 4 * math.ulp(r)
