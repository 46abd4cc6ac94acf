"""Pins of the pattern-prefix search oracle (paper Sec. 5, second
application): the suffix array and the per-query ranges against a textbook
example and brute force over every text position (no bisection, no sorted
list), and the query-record encoding against the string order."""
import numpy as np
import pytest

import oracle
from oracle import search_ref


def test_banana_textbook():
    # the classic example: suffixes of "banana" in order a, ana, anana,
    # banana, na, nana start at 5, 3, 1, 0, 4, 2
    text = b"banana"
    sa = search_ref.suffix_array(text)
    assert sa.tolist() == [5, 3, 1, 0, 4, 2]
    lo, hi = search_ref.prefix_ranges(text, sa, [b"an", b"na", b"ba", b"a\0", b"nb", b"aa", b"zz"], 2)
    assert list(zip(lo.tolist(), hi.tolist())) == [(1, 3), (4, 6), (3, 4), (0, 1), (6, 6), (1, 1), (6, 6)]


def brute(text: bytes, q: bytes, k: int):
    """(number of positions whose padded k-prefix is smaller than q, number equal)."""
    less = eq = 0
    for i in range(len(text)):
        p = text[i:i + k] + b"\0" * max(0, i + k - len(text))
        for a, b in zip(p, q):        # first differing character decides
            if a != b:
                less += a < b
                break
        else:
            eq += 1
    return less, eq


@pytest.mark.parametrize("alphabet,n,k", [(2, 50, 3), (4, 300, 4), (4, 1000, 8), (20, 500, 2), (4, 200, 16)])
def test_ranges_brute_force(alphabet, n, k, rng):
    text = bytes((rng.integers(0, alphabet, n) + 1).astype(np.uint8))
    sa = search_ref.suffix_array(text)
    # the array is a permutation whose suffixes increase, checked character by character
    assert sorted(sa.tolist()) == list(range(n))
    for a, b in zip(sa[:-1], sa[1:]):
        x, y = text[int(a):], text[int(b):]
        j = 0
        while j < len(x) and j < len(y) and x[j] == y[j]:
            j += 1
        assert j == len(x) or (j < len(y) and x[j] < y[j])
    qs = [text[int(i):int(i) + k].ljust(k, b"\0") for i in rng.integers(0, n, 40)]
    qs += [bytes((rng.integers(0, alphabet + 1, k) + 1).astype(np.uint8)) for _ in range(20)]
    lo, hi = search_ref.prefix_ranges(text, sa, qs, k)
    for q, a, b in zip(qs, lo, hi):
        less, eq = brute(text, q, k)
        assert (int(a), int(b) - int(a)) == (less, eq)


def test_query_records_follow_string_order(rng):
    k = 6
    qs = [bytes((rng.integers(0, 4, k) + 1).astype(np.uint8)) for _ in range(500)]
    rec = search_ref.query_records(qs, k, 16)
    assert search_ref.record_queries(rec, k) == qs
    out = oracle.sort(rec, k)
    got = search_ref.record_queries(out, k)
    assert got == sorted(qs)
    ids = out[:, k:k + 8].copy().view("<u8").ravel()
    assert [qs[int(i)] for i in ids] == got
