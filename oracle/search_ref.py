"""Batched pattern-prefix search over a suffix array -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product path never does.

The paper's second application (Sec. 5): many patterns are looked up in a
suffix array of a text (the text's suffixes in lexicographic order).  Each
pattern is searched for by binary search over the sorted suffixes; sorting
the patterns (or just their prefixes) first lets the searches run with
ranges narrowed by their neighbours.  What every search computes is fixed
by definition, whatever order the patterns come in:

* a text is a byte string whose characters are all non-zero; a character
  position past the end of the text reads as 0 (below every character);
* the k-prefix of suffix i is ``text[i:i+k]`` padded with zeros to k bytes;
* for a k-byte query q, ``lo`` = the number of suffixes whose k-prefix is
  smaller than q and ``hi`` = the number whose k-prefix is at most q, both
  compared as byte strings; ``sa[lo:hi]`` are then the suffixes that start
  with q.

A query travels as a record whose key (key_bytes = k, little-endian
integer) holds q reversed -- key byte k-1 is q's first character -- so that
the records' key order is q's string order.
"""
from __future__ import annotations

import bisect

import numpy as np


def suffix_array(text: bytes) -> np.ndarray:
    """Start positions of the suffixes in lexicographic order (definition)."""
    return np.array(sorted(range(len(text)), key=lambda i: text[i:]), dtype=np.uint32)


def k_prefix(text: bytes, i: int, k: int) -> bytes:
    return text[i:i + k] + b"\0" * max(0, i + k - len(text))


def prefix_ranges(text: bytes, sa: np.ndarray, queries, k: int):
    """(lo, hi) of each k-byte query (a bytes object), by bisection over the
    suffixes' k-prefixes listed in suffix-array order (sorted by definition of
    the suffix array)."""
    prefixes = [k_prefix(text, int(i), k) for i in sa]
    lo = np.array([bisect.bisect_left(prefixes, q) for q in queries], dtype=np.uint64)
    hi = np.array([bisect.bisect_right(prefixes, q) for q in queries], dtype=np.uint64)
    return lo, hi


def query_records(queries, k: int, rec_bytes: int, ids=None) -> np.ndarray:
    """Records of k-byte queries: key = the query reversed, then the query id
    (8 bytes, little-endian) if room, then zeros."""
    n = len(queries)
    rec = np.zeros((n, rec_bytes), dtype=np.uint8)
    for j, q in enumerate(queries):
        rec[j, :k] = np.frombuffer(q[::-1], dtype=np.uint8)
    if rec_bytes >= k + 8:
        ids = np.arange(n, dtype="<u8") if ids is None else np.asarray(ids, dtype="<u8")
        rec[:, k:k + 8] = ids.view(np.uint8).reshape(n, 8)
    return rec


def record_queries(rec: np.ndarray, k: int):
    """The k-byte queries held by query records (inverse of query_records)."""
    return [bytes(r[:k][::-1]) for r in rec]
