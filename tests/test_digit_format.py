"""Host checks of the integer format behind the WC projections (no GPU).

The chunked WC pass 1 forms <D[:, a], y[:, v]> on the matrix cores from 30-bit
fixed-point columns cut into four balanced 8-bit digits, sums the digit products
exactly in 32-bit integers grouped by weight 2^(8(i+j)), keeps the four classes
of weight 2^24 and above (C3..C6; the classes of weight 2^16 and below are
dropped), and combines C6*256 + C5 and C4*256 + C3 as two 32-bit halves before
one double FMA.  These tests restate that format in numpy and check the properties the
kernel relies on: digit ranges, exact recombination, no 32-bit overflow for
K <= 128 terms, and the size of the dropped part.
"""
import numpy as np
import pytest

K_MAX = 128          # 32 * k-steps, N_theta <= 128
Q_MAX = 1 << 30      # |q| <= 2^30 after scaling a column's largest magnitude into [2^29, 2^30)


def split(q):
    """Balanced base-256 digits (d0, d1, d2, d3) of int64 array q: d0..d2 in [-128, 127]."""
    q = np.asarray(q, dtype=np.int64).copy()
    out = []
    for _ in range(3):
        d = ((q + 128) & 255) - 128
        out.append(d)
        q = (q - d) >> 8
    out.append(q)
    return out


def classes(a, b):
    """S_ij summed over the K terms, grouped by weight i + j (16 classes, exact int64)."""
    da, db = split(a), split(b)
    c = np.zeros(7, dtype=np.int64)
    for i in range(4):
        for j in range(4):
            c[i + j] += int(np.dot(da[i], db[j]))
    return c


def test_digit_ranges_and_recombination():
    rng = np.random.default_rng(0)
    edge = np.array([0, 1, -1, 127, 128, -128, -129, 255, 256, -256, 32767, -32768,
                     Q_MAX, -Q_MAX, Q_MAX - 1, -(Q_MAX - 1), (1 << 29), -(1 << 29)], dtype=np.int64)
    q = np.concatenate([edge, rng.integers(-Q_MAX, Q_MAX + 1, 200000)])
    d0, d1, d2, d3 = split(q)
    for d in (d0, d1, d2):
        assert d.min() >= -128 and d.max() <= 127
    assert np.abs(d3).max() <= 64
    assert np.array_equal(d0 + 256 * (d1 + 256 * (d2 + 256 * d3)), q)


def test_classes_sum_to_the_exact_product():
    rng = np.random.default_rng(1)
    for k in (1, 32, 96, 128):
        a = rng.integers(-Q_MAX, Q_MAX + 1, k)
        b = rng.integers(-Q_MAX, Q_MAX + 1, k)
        c = classes(a, b)
        exact = sum(int(x) * int(y) for x, y in zip(a, b))
        assert sum(int(c[w]) << (8 * w) for w in range(7)) == exact


@pytest.mark.parametrize("sign", [1, -1])
def test_halves_fit_32_bits_at_the_worst_case(sign):
    # every digit product at its largest magnitude with one sign, K = 128 terms
    lo_digit, top = -128, 64
    a = [np.full(K_MAX, lo_digit)] * 3 + [np.full(K_MAX, top)]
    b = [np.full(K_MAX, sign * lo_digit)] * 3 + [np.full(K_MAX, sign * top)]
    c = np.zeros(7, dtype=np.int64)
    for i in range(4):
        for j in range(4):
            c[i + j] += int(np.dot(a[i], b[j]))
    c6, c5, c4, c3 = (int(c[w]) for w in (6, 5, 4, 3))
    assert abs(c6) <= 1 << 19 and abs(c5) <= 1 << 21 and abs(c4) <= 1 << 22 and abs(c3) < 3 << 21
    hi, lo = c6 * 256 + c5, c4 * 256 + c3
    assert abs(hi) < 1 << 31 and abs(lo) < 1 << 31
    kept = (hi << 16) + lo
    assert abs(kept) < 1 << 53            # exact in a double before the single rounding to float


def test_dropped_classes_at_the_worst_case():
    # classes of weight 2^16, 2^8, 2^0 with every digit product at its largest
    # magnitude: 3 K 2^30 + K 2^23 + K 2^14 against the largest sum K 2^60
    d = np.full(K_MAX, -128)
    c2, c1, c0 = 3 * int(np.dot(d, d)), 2 * int(np.dot(d, d)), int(np.dot(d, d))
    dropped = (c2 << 16) + (c1 << 8) + c0
    assert dropped / (K_MAX * Q_MAX * Q_MAX) < 3.01 * 2.0 ** -30


def test_dropped_classes_are_below_2_to_minus_29_of_the_largest_sum():
    rng = np.random.default_rng(2)
    largest = K_MAX * Q_MAX * Q_MAX
    worst = 0.0
    for _ in range(200):
        k = int(rng.integers(1, K_MAX + 1))
        a = rng.integers(-Q_MAX, Q_MAX + 1, k)
        b = rng.integers(-Q_MAX, Q_MAX + 1, k)
        c = classes(a, b)
        exact = sum(int(x) * int(y) for x, y in zip(a, b))
        kept = sum(int(c[w]) << (8 * w) for w in range(3, 7))
        worst = max(worst, abs(exact - kept) / largest)
    assert worst < 2.0 ** -29
