"""GPU parity: the HIP sort against the oracle, byte for byte."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import first_diff, note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1612_02557_amd import raduls
    assert torch.cuda.is_available()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    return raduls


def gpu_sort(R, host, k):
    import torch
    dev = to_dev(host)
    R.sort(dev, k)
    R.sync_check()
    torch.cuda.synchronize()
    return dev.cpu().numpy()


def check(R, host, k, label):
    note(label)
    got = gpu_sort(R, host, k)
    want = oracle.sort(host, k)
    assert np.array_equal(got, want), f"{label}: {first_diff(got, want)}"


SIZES = [2, 3, 31, 32, 33, 63, 64, 65, 100, 255, 256, 257, 1000, 2047, 2048, 2049, 4095, 4096, 4097,
         10000, 65535, 65536, 65537, 100_000, 1 << 20, 3_000_001]


@pytest.mark.parametrize("n", SIZES)
def test_uniform_16_8_sizes(R, n):
    host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=8, dist="uniform", seed=1))
    check(R, host, 8, f"uniform r=16 k=8 n={n}")


@pytest.mark.parametrize("dist", ["zipf", "prefix", "mix"])
@pytest.mark.parametrize("n", [5000, 200_000, 2_000_003])
def test_distributions(R, dist, n):
    host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=8, dist=dist, seed=3))
    check(R, host, 8, f"{dist} r=16 k=8 n={n}")


@pytest.mark.parametrize("r,k", [(8, 8), (16, 16), (32, 8), (32, 16), (4, 1), (4, 4), (12, 3), (20, 5),
                                 (64, 16), (24, 16), (8, 2), (48, 12), (60, 9)])
@pytest.mark.parametrize("n", [777, 70_001, 1_000_000])
def test_record_shapes(R, r, k, n):
    dist = "uniform" if k in (8, 16) else "bytes"
    host = synth.generate(synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=dist, payload="random", seed=5))
    check(R, host, k, f"{dist} r={r} k={k} n={n}")


@pytest.mark.parametrize("r,k", [(16, 16), (32, 16)])
@pytest.mark.parametrize("dist", ["zipf", "prefix", "mix"])
def test_wide_keys_skewed(R, r, k, dist):
    host = synth.generate(synth.Spec(n=300_000, rec_bytes=r, key_bytes=k, dist=dist, payload="random", seed=8))
    check(R, host, k, f"{dist} r={r} k={k} n=300000")


def _records_with_keys(keys, r=16):
    n = len(keys)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, :8] = np.asarray(keys, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("n", [50, 5000, 300_000])
def test_adversarial(R, n, rng):
    cases = {
        "all_equal": np.full(n, 0xDEADBEEF, dtype=np.uint64),
        "sorted": np.sort(rng.integers(0, 2**63, n, dtype=np.uint64)),
        "reverse": np.sort(rng.integers(0, 2**63, n, dtype=np.uint64))[::-1].copy(),
        "two_values": rng.choice(np.array([3, 2**63 + 5], dtype=np.uint64), n),
        "prefix56": (np.uint64(0xABCDEF12345678) << np.uint64(8)) | rng.integers(0, 256, n, dtype=np.uint64),
        "prefix40": (np.uint64(0xABCDEF1234) << np.uint64(24)) | rng.integers(0, 2**24, n, dtype=np.uint64),
        "low_bits_only": rng.integers(0, 16, n, dtype=np.uint64),
        "one_giant": np.where(rng.random(n) < 0.9, np.uint64(77), rng.integers(0, 2**64 - 1, n, dtype=np.uint64)),
        "max_keys": np.full(n, 2**64 - 1, dtype=np.uint64) - rng.integers(0, 3, n, dtype=np.uint64),
    }
    for name, keys in cases.items():
        check(R, _records_with_keys(keys), 8, f"adversarial {name} n={n}")


def _wide_records(hi, lo, r=32):
    n = len(hi)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, :8] = np.asarray(lo, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.asarray(hi, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 16:24] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("sched", ["heuristic", "RADIX"])
@pytest.mark.parametrize("n", [5000, 300_000])
def test_wide_keys_split_varying_bits(R, n, sched, rng):
    """16-byte keys whose varying bits sit at both ends of the key: the
    in-LDS radix composite keeps only the top varying bits, so keys that tie
    there and differ in the low bits (and exact duplicates) test the full-key
    tie rule."""
    const_hi, const_lo = np.uint64(0x0123456789ABCDEF), np.uint64(0xFEDCBA9876543210)
    cases = {}
    for top, low in ((4, 3), (6, 6), (10, 8), (16, 1)):
        hi = (rng.integers(0, 1 << top, n, dtype=np.uint64) << np.uint64(64 - top)) | (const_hi >> np.uint64(top))
        lo = ((const_lo >> np.uint64(low)) << np.uint64(low)) | rng.integers(0, 1 << low, n, dtype=np.uint64)
        cases[f"top{top}_low{low}"] = (hi, lo)
    if sched == "RADIX":
        R.set_scheduler(R.SCHED_FORCED, R.PROC_RADIX)
    try:
        for name, (hi, lo) in cases.items():
            check(R, _wide_records(hi, lo), 16, f"wide split {name} n={n} {sched}")
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)


def test_empty_and_single(R):
    import torch
    for n in (0, 1):
        note(f"n={n}")
        host = synth.generate(synth.Spec(n=max(n, 1), rec_bytes=16, key_bytes=8, seed=2))[:n]
        dev = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
        if n:
            dev.copy_(to_dev(host))
        R.sort(dev, 8)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy(), host)


@pytest.mark.parametrize("proc", ["RADIX", "LSD", "BITONIC"])
@pytest.mark.parametrize("dist", ["uniform", "zipf", "mix"])
def test_forced_procedures_same_bytes(R, proc, dist):
    host = synth.generate(synth.Spec(n=400_000, rec_bytes=16, key_bytes=8, dist=dist, seed=13))
    p = {"RADIX": R.PROC_RADIX, "LSD": R.PROC_LSD, "BITONIC": R.PROC_BITONIC}[proc]
    R.set_scheduler(R.SCHED_FORCED, p)
    try:
        check(R, host, 8, f"forced {proc} {dist} n=400000")
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)


TUNINGS = [
    dict(big_digit_bits=4),
    dict(big_digit_bits=6, block_digit_bits=5),
    dict(big_digit_bits=11),
    dict(block_digit_bits=3, lds_finish_max=256, bitonic_max=64),
    dict(tile_records=256, big_min=4096),
    dict(tile_records=1024, big_min=2048, workgroups_per_cu=1),
    dict(nontemporal=1, workgroups_per_cu=4),
    dict(reg_finish=0),
    dict(reg_finish=0, big_digit_bits=6, job_records=512),
    dict(reg_finish=1, job_records=4096),
    dict(reg_finish=1, big_digit_bits=11, tile_records=2048, big_min=4096),
]


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_tuning_invariance(R, ti):
    host = synth.generate(synth.Spec(n=500_000, rec_bytes=16, key_bytes=8, dist="mix", seed=21))
    t = R.default_tuning(16, 8, 500_000)
    for kk, v in TUNINGS[ti].items():
        setattr(t, kk, v)
    R.set_tuning(t)
    try:
        check(R, host, 8, f"tuning {TUNINGS[ti]}")
    finally:
        R.set_tuning(None)


def test_run_twice_identical(R):
    host = synth.generate(synth.Spec(n=1_000_000, rec_bytes=16, key_bytes=8, dist="mix", seed=4))
    note("run twice")
    a = gpu_sort(R, host, 8)
    b = gpu_sort(R, host, 8)
    assert np.array_equal(a, b)


def _dup_records(keys, r=16):
    n = len(keys)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, 0:8] = np.asarray(keys, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("case", ["three_keys", "heavy_key", "low_bits", "high_bits", "two_heavy"])
def test_register_finish_duplicates(R, case, rng):
    """Jobs of the register-finishing kernel whose digit sub-bins are large
    (runs of equal keys, few varying bits): the wavefront bitonic network and
    the binary-search slots, against the oracle."""
    if case == "three_keys":
        keys = rng.choice(np.array([5, 1 << 40, (1 << 63) + 7], dtype=np.uint64), 300_000)
    elif case == "heavy_key":
        keys = rng.integers(0, 1 << 64, 20_000, dtype=np.uint64)
        keys[rng.random(20_000) < 0.75] = np.uint64(0x0123456789ABCDEF)
    elif case == "low_bits":
        keys = np.uint64(0xABCDEF0000000000) | rng.integers(0, 1 << 9, 200_000, dtype=np.uint64)
    elif case == "high_bits":
        keys = rng.integers(0, 1 << 10, 200_000, dtype=np.uint64) << np.uint64(54)
    else:
        keys = rng.integers(0, 1 << 64, 16_000, dtype=np.uint64)
        u = rng.random(16_000)
        keys[u < 0.4] = np.uint64(3)
        keys[u > 0.6] = np.uint64(3) + np.uint64(1 << 20)
    check(R, _dup_records(keys), 8, f"register finish {case} n={len(keys)}")


def _dup_records16(hi, lo, r=32):
    n = len(hi)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, 0:8] = np.asarray(lo, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.asarray(hi, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 16:24] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("case", ["kmer_like", "heavy_key", "low_word_only", "high_word_only", "straddle"])
def test_register_finish_wide_keys(R, case, rng):
    """Jobs of 16-byte keys finished with 128-bit composites: runs of equal
    keys, keys that differ only in the low or only in the high word, and
    varying bits on both sides of the word boundary, against the oracle."""
    n = 300_000
    if case == "kmer_like":       # few distinct random keys, many copies of each
        pool_hi = rng.integers(0, 1 << 64, 3000, dtype=np.uint64)
        pool_lo = rng.integers(0, 1 << 64, 3000, dtype=np.uint64)
        j = rng.integers(0, 3000, n)
        hi, lo = pool_hi[j], pool_lo[j]
    elif case == "heavy_key":
        hi = rng.integers(0, 1 << 64, n, dtype=np.uint64)
        lo = rng.integers(0, 1 << 64, n, dtype=np.uint64)
        heavy = rng.random(n) < 0.6
        hi[heavy], lo[heavy] = np.uint64(0x0123456789ABCDEF), np.uint64(0xFEDCBA9876543210)
    elif case == "low_word_only":
        hi = np.full(n, 0xABCDEF0123456789, dtype=np.uint64)
        lo = rng.integers(0, 1 << 64, n, dtype=np.uint64)
    elif case == "high_word_only":
        hi = rng.integers(0, 1 << 64, n, dtype=np.uint64)
        lo = np.full(n, 77, dtype=np.uint64)
    else:                         # 20 varying bits around bit 64
        v = rng.integers(0, 1 << 20, n, dtype=np.uint64)
        hi = np.uint64(0x5555000000000000) | (v >> np.uint64(10))
        lo = np.uint64(0x00000000000000FF) | ((v & np.uint64(1023)) << np.uint64(54))
    check(R, _dup_records16(hi, lo), 16, f"register finish wide {case} n={n}")
