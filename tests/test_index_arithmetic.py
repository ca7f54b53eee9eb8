"""Host checks of the integer arithmetic the particle kernel relies on.

The kernel decodes node and row indexes of its block box by
floor((n + 1/2) * r) with r = 1/d rounded to FP64, instead of an integer
division, and divides cell indexes by the sort-tile dims with a 32-bit
multiply-high by ceil(2^32 / d).  Both are exact only on a range; these
tests check them on every value the kernel can meet (box volumes up to four
times the 1650-node LDS box, row counts of a block box in a 2^20-node
grid), with IEEE double arithmetic as on the device.
"""
import numpy as np


def small_div(n, d):
    inv = 1.0 / np.float64(d)
    return np.floor((n.astype(np.float64) + 0.5) * inv).astype(np.int64)


def test_reciprocal_division_is_exact_on_the_box_range():
    n = np.arange(4 * 1650, dtype=np.int64)
    for d in range(1, 1651):
        np.testing.assert_array_equal(small_div(n, d), n // d, err_msg=f"d={d}")


def test_reciprocal_division_is_exact_for_large_row_counts():
    rng = np.random.default_rng(7)
    d = rng.integers(1, 1 << 20, size=200_000)
    n = rng.integers(0, 1 << 40, size=200_000)
    q = np.floor((n.astype(np.float64) + 0.5) * (1.0 / d.astype(np.float64))).astype(np.int64)
    np.testing.assert_array_equal(q, n // d)
    # the worst case of the rounding argument: n + 1/2 just past a multiple of d
    d = np.arange(1, 1 << 14, dtype=np.int64)
    for k in (1, 3, 1 << 10, (1 << 26) - 1):
        for off in (-1, 0):
            n = k * d + off
            ok = n >= 0
            q = np.floor((n[ok].astype(np.float64) + 0.5) * (1.0 / d[ok].astype(np.float64))).astype(np.int64)
            np.testing.assert_array_equal(q, n[ok] // d[ok])


def _mulhi_div(t, d):
    m = 0 if d == 1 else (0xFFFFFFFF // d + 1)
    if d == 1:
        return t
    return (t.astype(np.uint64) * np.uint64(m)) >> np.uint64(32)


def test_multiply_high_tile_division_is_exact():
    # cells below 2^20, tile dims 1..64 (the descriptor's limits)
    t = np.concatenate([np.arange(1 << 16, dtype=np.uint64),
                        np.random.default_rng(3).integers(0, 1 << 20, size=100_000).astype(np.uint64),
                        np.arange((1 << 20) - 4096, 1 << 20, dtype=np.uint64)])
    for d in range(1, 65):
        np.testing.assert_array_equal(_mulhi_div(t, d), t // np.uint64(d), err_msg=f"d={d}")
