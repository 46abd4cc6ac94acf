"""Heuristic procedure rules and regret (TEST INFRASTRUCTURE ONLY).

The paper's scheduler (Sec. 3.2-3.5) picks, per bin, how to process it from
its size alone, with constants it chose by experiment:
  * a bin is big, and gets a multi-thread pass, when it holds more than
    2N/(3T) records (N all records, T threads), Sec. 3.2;
  * every other bin gets another radix pass; one that fits in half of the
    L2 cache is split by a plain counting pass in cache, a larger one by the
    buffered split, Sec. 3.4;
  * a bin with fewer than 384 keys is finished by a comparison sort; when the
    narrowing factor (parent size / bin size) exceeds sqrt(R) = 16 that tiny
    threshold drops to 32; insertion sort serves bins of at most 32, Sec. 3.5.

``heuristic`` restates those rules over the GPU procedures, reading "threads"
as concurrently resident workgroups and "fits in cache" as "fits the
workgroup's local data share":
  RANK     (one wavefront, all-pairs rank; the insertion-sort slot)  m <= 32
  BITONIC  (comparison sort in LDS)             m < tiny(m, parent)
  RADIX    (one more radix pass: inside LDS when m <= lds_capacity, its
            sub-bins insertion sorted; through memory otherwise)
and BIG (multi-workgroup pass) for m > 2N/(3W).  LSD (stable counting passes
inside LDS) is a further procedure that only the learned or forced
scheduler picks.
"""
from __future__ import annotations

import math

PROC_RADIX, PROC_LSD, PROC_BITONIC = 0, 1, 2
PROC_RANK, PROC_BIG, PROC_DONE = 3, 4, 5
N_CHOICES = 3          # procedures the learned scheduler chooses between

TINY = 384             # Sec. 3.5
TINY_NARROW = 32       # Sec. 3.5, when the narrowing factor exceeds 16
NARROW = 16            # sqrt(R) with R = 256, Sec. 3.5
INSERTION_MAX = 32     # Sec. 3.5


def big_threshold(N: int, W: int, floor: int) -> int:
    """Records above which a bucket is big: 2N/(3W), Sec. 3.2 (not below ``floor``)."""
    return max(2 * N // (3 * W), floor)


def heuristic(m: int, parent_m: int, bits_left: int, lds_capacity: int, bitonic_capacity: int,
              big: int) -> int:
    """Procedure for a bucket of m records whose parent held parent_m."""
    if m <= 1 or bits_left <= 0:
        return PROC_DONE
    if m > big:
        return PROC_BIG
    if m <= INSERTION_MAX:
        return PROC_RANK
    narrowing = parent_m / m
    tiny = TINY_NARROW if narrowing > NARROW else TINY
    if m < tiny and m <= bitonic_capacity:
        return PROC_BITONIC
    return PROC_RADIX


def features(m: int, parent_m: int, bit: int, key_bits: int, rec_bytes: int, key_bytes: int):
    """The nine scheduler-network inputs of a bucket (all float)."""
    lm = math.log2(m)
    lp = math.log2(max(parent_m, m))
    return [
        lm,
        lp,
        lp - lm,
        (key_bits - bit) / 64.0,
        bit / 64.0,
        rec_bytes / 64.0,
        key_bytes / 16.0,
        math.log2(m * rec_bytes) - 16.0,
        1.0 if (lp - lm) > 4.0 else 0.0,
    ]


def regret(chosen, times) -> float:
    """sum_b [t_b(chosen_b) - min_p t_b(p)] / sum_b min_p t_b(p).

    ``times`` is a list of per-bucket sequences with None (or NaN) for
    procedures not observed; ``chosen`` holds each bucket's chosen index.
    """
    num = 0.0
    den = 0.0
    for c, t in zip(chosen, times):
        obs = [x for x in t if x is not None and not math.isnan(x)]
        if not obs:
            continue
        best = min(obs)
        tc = t[c]
        if tc is None or math.isnan(tc):
            raise ValueError("chosen procedure has no observed time")
        num += tc - best
        den += best
    return num / den if den > 0 else 0.0
