"""The library's stable radix sort and exclusive scan (the binning of
constraint rows by cell, the data-node slots and the marching-cubes offsets)
against numpy's stable argsort and cumulative sum, bit for bit: ragged sizes
around the 1024-row blocks and 64-row chunks, heavy ties, every digit-pass
count, all-equal keys, keys of the full 32 bits, and the sizes of the 64^3
workload."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _check_sort(keys, end_bit):
    from paper_1603_08161_amd import sort_pairs
    vals = np.arange(keys.size, dtype=np.int32)[::-1].copy()  # distinct, not the row order
    ko, vo = sort_pairs(keys, vals, end_bit)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(ko, keys[order])
    np.testing.assert_array_equal(vo, vals[order])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1023, 1024, 1025, 4097, 65536 + 7])
@pytest.mark.parametrize("end_bit", [1, 8, 9, 16, 18])
def test_sort_is_stable_and_ordered(n, end_bit):
    rng = np.random.default_rng(n * 131 + end_bit)
    hi = min(1 << end_bit, max(2, n // 3))  # many ties
    keys = rng.integers(0, hi, size=n).astype(np.uint32)
    _check_sort(keys, end_bit)


def test_sort_edge_cases():
    from paper_1603_08161_amd import sort_pairs
    rng = np.random.default_rng(7)
    _check_sort(np.zeros(3000, np.uint32), 1)                            # all equal
    _check_sort(np.full(5000, 0x3FFFF, np.uint32), 18)                   # all equal, top digit
    _check_sort(rng.integers(0, 2**32, size=20000, dtype=np.uint64).astype(np.uint32), 32)
    _check_sort(np.arange(9000, dtype=np.uint32)[::-1].copy(), 14)      # reversed
    _check_sort(np.zeros(100, np.uint32), 0)                             # no pass: a copy
    ko, vo = sort_pairs(np.zeros(0, np.uint32), np.zeros(0, np.int32), 8)
    assert ko.size == 0 and vo.size == 0


def test_sort_rows_of_the_64cubed_workload():
    """About 108k rows (dense samples + 3 per sparse pair) on 63^3 cells, as
    the finest level bins them."""
    rng = np.random.default_rng(11)
    cells = 63 ** 3
    hot = rng.integers(0, cells, size=6000)
    keys = hot[rng.integers(0, hot.size, size=108662)].astype(np.uint32)
    _check_sort(keys, int(np.ceil(np.log2(cells))))


@pytest.mark.parametrize("n", [1, 255, 256, 1023, 1024, 1025, 262144, 884736, 1024 * 1024 + 3])
def test_exclusive_scan(n):
    from paper_1603_08161_amd import exclusive_scan
    rng = np.random.default_rng(n)
    x = rng.integers(0, 6, size=n).astype(np.int32)
    out = exclusive_scan(x)
    ref = np.concatenate([[0], np.cumsum(x, dtype=np.int64)[:-1]]).astype(np.int32)
    np.testing.assert_array_equal(out, ref)
