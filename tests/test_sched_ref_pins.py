"""Pins of the heuristic rules and the regret measure (``oracle.sched_ref``)."""
import math
import os

import pytest

from oracle import sched_ref as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def paper_constants():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value = line.split()[:2]
            out[name] = int(value)
    return out


def test_constants_are_the_papers():
    c = paper_constants()
    assert S.TINY == c["tiny_bin"]
    assert S.TINY_NARROW == c["tiny_bin_narrow"]
    assert S.NARROW == c["narrowing_factor"] == int(math.isqrt(c["radix"]))
    assert S.INSERTION_MAX == c["insertion_max"]
    N, W = 3_000_000, 100
    assert S.big_threshold(N, W, 0) == c["big_bin_numerator"] * N // (c["big_bin_denominator"] * W)


def test_rule_boundaries():
    big, lds, bit = 1 << 20, 4096, 4096
    h = lambda m, p: S.heuristic(m, p, 40, lds, bit, big)
    assert h(1, 100) == S.PROC_DONE
    assert S.heuristic(50, 100, 0, lds, bit, big) == S.PROC_DONE
    assert h(32, 64) == S.PROC_RANK            # insertion-sort slot: N <= 32
    assert h(33, 66) == S.PROC_BITONIC         # tiny: fewer than 384 keys
    assert h(383, 766) == S.PROC_BITONIC
    assert h(384, 768) == S.PROC_RADIX         # not tiny any more (strict "<")
    # narrowing factor above 16 lowers the tiny threshold to 32
    assert h(100, 1601) == S.PROC_RADIX
    assert h(100, 1600) == S.PROC_BITONIC      # exactly 16 is not "larger than"
    assert h(4096, 10**6) == S.PROC_RADIX      # in LDS
    assert h(4097, 10**6) == S.PROC_RADIX      # through memory
    assert h(big, 10**9) == S.PROC_RADIX
    assert h(big + 1, 10**9) == S.PROC_BIG


def test_regret_hand_example():
    times = [[3.0, 1.0, 2.0], [5.0, None, 4.0], [2.0, 2.0, float("nan")]]
    # best: 1, 4, 2 (sum 7); chosen 0, 2, 1 -> 3 + 4 + 2 = 9 -> regret 2/7
    assert S.regret([0, 2, 1], times) == pytest.approx(2.0 / 7.0)
    assert S.regret([1, 2, 0], times) == 0.0
    with pytest.raises(ValueError):
        S.regret([1], [[1.0, None, 2.0]])


def test_features_shape_and_values():
    f = S.features(1024, 65536, 16, 64, 16, 8)
    assert len(f) == 9
    assert f[0] == 10 and f[1] == 16 and f[2] == 6 and f[8] == 1.0
    assert f[3] == 48 / 64 and f[4] == 16 / 64 and f[7] == 14 - 16 + 0.0


def test_learn_regret_matches_reference():
    """The training module's vectorised regret equals the reference definition."""
    import numpy as np
    from paper_1612_02557_amd import learn
    rng = np.random.default_rng(5)
    n = 200
    feas = rng.integers(1, 8, n).astype(np.uint32)
    ticks = rng.integers(1, 10_000, (n, 3)).astype(np.uint32)
    chosen = np.array([rng.choice([q for q in range(3) if (f >> q) & 1]) for f in feas])
    times = [[float(ticks[i, q]) if (feas[i] >> q) & 1 else None for q in range(3)] for i in range(n)]
    assert learn.regret(chosen, ticks, feas) == pytest.approx(S.regret(list(chosen), times))
