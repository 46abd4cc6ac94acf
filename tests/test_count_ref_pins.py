"""Pins of the duplicate-removal oracle (k-mer counting application, paper
Sec. 5: sort the k-mers, then remove duplicates keeping a count).

``oracle.sort_count`` is checked against ``collections.Counter`` over keys
decoded by ``int.from_bytes`` (a hash table instead of a scan of sorted
runs), the first record of each key found by brute force over the input
(the earliest input index, which a stable sort puts first), closed forms
(all keys equal, all keys distinct, empty and single inputs) and the
invariants (counts sum to n, unique keys strictly increasing)."""
import collections
import itertools

import numpy as np
import pytest

import oracle


def counter_reference(rec: np.ndarray, k: int):
    keys = [int.from_bytes(bytes(x[:k]), "little") for x in rec]
    cnt = collections.Counter(keys)
    first = {}
    for i, key in enumerate(keys):
        first.setdefault(key, i)
    order = sorted(cnt)
    uniq = np.array([rec[first[key]] for key in order], dtype=np.uint8).reshape(len(order), rec.shape[1])
    return uniq, np.array([cnt[key] for key in order], dtype=np.uint64)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_exhaustive_small_alphabet(n):
    for keys in itertools.product(range(3), repeat=n):
        rec = np.zeros((n, 4), dtype=np.uint8)
        rec[:, 0] = keys
        rec[:, 1] = np.arange(n)
        u, c = oracle.sort_count(rec, 1)
        wu, wc = counter_reference(rec, 1)
        np.testing.assert_array_equal(u, wu)
        np.testing.assert_array_equal(c, wc)


@pytest.mark.parametrize("k,r", [(1, 4), (2, 8), (3, 12), (8, 8), (8, 16), (12, 20), (16, 16), (16, 32)])
def test_random_vs_counter(k, r, rng):
    for n, alphabet in ((50, 4), (700, 30), (3000, 3000)):
        rec = rng.integers(0, 256, size=(n, r), dtype=np.uint8)
        # keys from a small set of byte patterns; pairs that differ only in the
        # most significant key byte, or only in the least significant one
        pats = rng.integers(0, 256, size=(alphabet, k), dtype=np.uint8)
        if alphabet >= 4:
            pats[1] = pats[0]
            pats[1, k - 1] ^= 0x80
            pats[2] = pats[0]
            pats[2, 0] ^= 1
        rec[:, :k] = pats[rng.integers(0, alphabet, n)]
        u, c = oracle.sort_count(rec, k)
        wu, wc = counter_reference(rec, k)
        np.testing.assert_array_equal(u, wu)
        np.testing.assert_array_equal(c, wc)


def test_closed_forms(rng):
    n, r = 1000, 16
    rec = rng.integers(0, 256, size=(n, r), dtype=np.uint8)
    # all keys equal: one run, its first record is the first input record
    same = rec.copy()
    same[:, :8] = rec[0, :8]
    u, c = oracle.sort_count(same, 8)
    np.testing.assert_array_equal(u, same[:1])
    np.testing.assert_array_equal(c, [n])
    # all keys distinct: every record is its own run, in sorted order
    distinct = rec.copy()
    distinct[:, :8] = np.frombuffer(rng.permutation(np.arange(n, dtype="<u8") * 7919).tobytes(),
                                    dtype=np.uint8).reshape(n, 8)
    u, c = oracle.sort_count(distinct, 8)
    np.testing.assert_array_equal(u, oracle.sort(distinct, 8))
    assert np.all(c == 1)
    # empty and single inputs
    u, c = oracle.sort_count(rec[:0], 8)
    assert u.shape == (0, r) and c.shape == (0,)
    u, c = oracle.sort_count(rec[:1], 8)
    np.testing.assert_array_equal(u, rec[:1])
    np.testing.assert_array_equal(c, [1])


def test_invariants(rng):
    n, r, k = 20000, 16, 16
    rec = rng.integers(0, 256, size=(n, r), dtype=np.uint8)
    rec[:, :k] = rec[rng.integers(0, 2000, n), :k]
    u, c = oracle.sort_count(rec, k)
    assert int(c.sum()) == n
    keys = [int.from_bytes(bytes(x[:k]), "little") for x in u]
    assert all(a < b for a, b in zip(keys, keys[1:]))
