"""The one-pair-per-thread enumeration of the Lennard-Jones pairs in the
paper's energy routine (Sec. 3.4), as the pair-per-thread energy kernel takes
it: in round i = 0 .. floor(N/2) - 1 thread v takes (i, v) when v > i, else
(N-2-i, N-1-i+v).  Read as printed, the guard i != N-2-i drops the whole
middle round for even N, and with it every pair of row N/2 - 1; taking only
the threads v > i in that round covers every pair exactly once."""
from collections import Counter

import pytest


def enumerate_pairs(n, fixed=True):
    out = []
    for i in range(n // 2):
        middle = n - 2 - i == i
        if middle and not fixed:
            continue  # the printed guard: the whole round is skipped
        for v in range(n):
            if v > i:
                out.append((i, v))
            elif not middle:
                out.append((n - 2 - i, n - 1 - i + v))
    return out


@pytest.mark.parametrize("n", list(range(2, 81)))
def test_fixed_enumeration_covers_every_pair_once(n):
    got = Counter(enumerate_pairs(n))
    want = Counter((i, j) for i in range(n) for j in range(i + 1, n))
    assert got == want


@pytest.mark.parametrize("n", list(range(2, 81)))
def test_printed_guard_drops_the_middle_row_for_even_n(n):
    got = set(enumerate_pairs(n, fixed=False))
    want = {(i, j) for i in range(n) for j in range(i + 1, n)}
    missing = want - got
    if n % 2:
        assert not missing
    else:
        assert missing == {(n // 2 - 1, j) for j in range(n // 2, n)}
