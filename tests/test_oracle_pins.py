"""Pins of the sorting oracle against things other than itself.

* Python's built-in ``sorted`` (Timsort, documented stable) with an integer
  key built by ``int.from_bytes`` -- a different algorithm and a different
  key decoder -- exhaustively on tiny inputs and randomly on larger ones;
* closed-form special cases (sorted, all-equal, reversed distinct keys,
  one-byte keys = numpy's stable argsort);
* the LSD-radix composition theorem with digit widths other than the
  oracle's bytes (4, 11, 16 bits), through the one-digit partition;
* invariants: keys non-decreasing, output a permutation of the input.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def py_stable_sort(rec: np.ndarray, k: int) -> np.ndarray:
    rows = [bytes(x) for x in rec]
    rows_sorted = sorted(rows, key=lambda b: int.from_bytes(b[:k], "little"))
    return np.frombuffer(b"".join(rows_sorted), dtype=np.uint8).reshape(rec.shape)


def keys_int(rec: np.ndarray, k: int):
    return [int.from_bytes(bytes(x[:k]), "little") for x in rec]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_exhaustive_small_alphabet(n):
    # every key sequence over {0, 1, 2}; payload = index (so ties are visible)
    for keys in itertools.product(range(3), repeat=n):
        rec = np.zeros((n, 4), dtype=np.uint8)
        for i, key in enumerate(keys):
            rec[i, 0] = key
            rec[i, 1] = i
        np.testing.assert_array_equal(oracle.sort(rec, 1), py_stable_sort(rec, 1))


@pytest.mark.parametrize("k,r", [(1, 1), (1, 4), (2, 2), (2, 8), (3, 7), (3, 16), (8, 8), (8, 12),
                                 (8, 16), (8, 32), (16, 16), (16, 20), (16, 32)])
def test_random_vs_python_sorted(k, r, rng):
    for n in (7, 100, 4096):
        rec = rng.integers(0, 256, size=(n, r), dtype=np.uint8)
        if k > 1:  # force many ties on the high bytes too
            rec[: n // 2, k - 1] = 0
        np.testing.assert_array_equal(oracle.sort(rec, k), py_stable_sort(rec, k))


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threads_identical(threads, rng):
    rec = rng.integers(0, 256, size=(5000, 16), dtype=np.uint8)
    rec[:, 3:8] = 0
    np.testing.assert_array_equal(oracle.sort_threads(rec, 8, threads), oracle.sort(rec, 8))


def test_special_cases(rng):
    n, r, k = 3000, 16, 8
    # already sorted distinct keys -> identity
    keys = np.sort(rng.choice(2**62, size=n, replace=False)).astype("<u8")
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, :8] = keys.view(np.uint8).reshape(n, 8)
    rec[:, 8:] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    np.testing.assert_array_equal(oracle.sort(rec, k), rec)
    # reversed distinct keys -> exact reversal
    rev = rec[::-1].copy()
    np.testing.assert_array_equal(oracle.sort(rev, k), rec)
    # all keys equal -> identity (stability)
    same = rec.copy()
    same[:, :8] = 7
    np.testing.assert_array_equal(oracle.sort(same, k), same)
    # one-byte key -> numpy's stable argsort of that byte
    one = rng.integers(0, 256, size=(n, 8), dtype=np.uint8)
    order = np.argsort(one[:, 0], kind="stable")
    np.testing.assert_array_equal(oracle.sort(one, 1), one[order])


def test_invariants_on_generated_inputs():
    for dist in ("uniform", "zipf", "prefix", "mix"):
        for (r, k) in ((8, 8), (16, 8), (16, 16), (32, 8), (32, 16)):
            rec = synth.generate(synth.Spec(n=20000, rec_bytes=r, key_bytes=k, dist=dist,
                                            payload="random", seed=7))
            out = oracle.sort(rec, k)
            ks = keys_int(out, k)
            assert all(a <= b for a, b in zip(ks, ks[1:]))
            a = np.sort(rec.view(np.dtype((np.void, r))).ravel())
            b = np.sort(out.view(np.dtype((np.void, r))).ravel())
            assert (a == b).all()


@pytest.mark.parametrize("bits", [4, 11, 16])
def test_lsd_composition_with_other_digit_widths(bits):
    # the LSD theorem: stable partitions on successive digits, least
    # significant first, sort the array; digits here are not the oracle's bytes
    rec = synth.generate(synth.Spec(n=3000, rec_bytes=16, key_bytes=8, dist="zipf",
                                    payload="index", seed=11, zipf_m=500))
    cur = rec
    for shift in range(0, 64, bits):
        cur = oracle.partition(cur, 8, shift, min(bits, 64 - shift))
    np.testing.assert_array_equal(cur, oracle.sort(rec, 8))


@pytest.mark.parametrize("k,shift,bits", [(8, 56, 8), (8, 0, 11), (8, 60, 8), (16, 100, 9),
                                          (16, 120, 8), (3, 4, 16)])
def test_partition_and_histogram_vs_python(k, shift, bits, rng):
    r = 16 if k <= 16 else k
    rec = rng.integers(0, 256, size=(2000, r), dtype=np.uint8)
    dig = [(v >> shift) & ((1 << bits) - 1) for v in keys_int(rec, k)]
    order = sorted(range(len(rec)), key=lambda i: dig[i])   # stable
    np.testing.assert_array_equal(oracle.partition(rec, k, shift, bits), rec[order])
    h = oracle.digit_histogram(rec, k, shift, bits)
    np.testing.assert_array_equal(h, np.bincount(dig, minlength=1 << bits))
    assert int(h.sum()) == len(rec)


def test_segments_each_sorted(rng):
    sizes = np.array([0, 1, 5, 300, 2, 1000], dtype=np.uint64)
    off = synth.segment_offsets(sizes)
    rec = rng.integers(0, 256, size=(int(off[-1]), 16), dtype=np.uint8)
    out = oracle.sort_segments(rec, off, 8)
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        np.testing.assert_array_equal(out[a:b], py_stable_sort(rec[a:b], 8))


def test_rejects_bad_arguments():
    rec = np.zeros((4, 8), dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.sort(rec, 0)
    with pytest.raises(ValueError):
        oracle.sort(rec, 9)
