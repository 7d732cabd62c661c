"""The bench's flop accounting for the symmetric dense product, checked against a brute-force count of
the entries of A that the library's row tiles multiply by Z (2 n flops per entry).  The dominant
kernel's roofline fraction divides these flops by its launch time, so a miscount there would misstate
it.  Host arithmetic only."""
import numpy as np
import pytest

import bench


def _block_mask(m, bm, diag):
    """Entries (i, k) of A read by the product: row tile t = i // bm takes K from its own diagonal block
    (diag) or from the block right of it."""
    i = np.arange(m)[:, None]
    k = np.arange(m)[None, :]
    start = (i // bm + (0 if diag else 1)) * bm
    return k >= start


@pytest.mark.parametrize("m,n,bm", [(64, 3, 64), (65, 5, 64), (300, 7, 64), (1000, 16, 64), (257, 2, 32)])
def test_upper_product_flops_counts_the_multiplied_entries(m, n, bm):
    for diag in (False, True):
        expected = 2.0 * n * int(_block_mask(m, bm, diag).sum())
        assert bench.upper_product_flops(m, n, bm, diag=diag) == expected


def test_diagonal_blocks_add_their_own_products():
    # W' = (U + D/2) Z computes every diagonal block in full (its lower triangle as zeros): the
    # difference between the two counts is 2 n sum of the squared tile heights
    m, n, bm = 1000, 16, 64
    rows = [min(bm, m - t) for t in range(0, m, bm)]
    diff = bench.upper_product_flops(m, n, bm, diag=True) - bench.upper_product_flops(m, n, bm)
    assert diff == 2.0 * n * sum(r * r for r in rows)


def test_symmetric_pass_is_about_half_of_the_full_product():
    # reading the upper block triangle halves the 2 m^2 n of A Z, up to the diagonal blocks
    m, n = 32768, 256
    full = 2.0 * m * m * n
    up = bench.upper_product_flops(m, n, diag=True)
    assert 0.5 * full < up < 0.5 * full + 2.0 * 64 * m * n + 1
