"""GPU parity of the in-place sort (``raduls_sort_inplace``): the keys of
the output are the oracle's, byte for byte, and the output records are a
permutation of the input (the in-place variant is not stable, so records
with equal keys may come in any order)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import note, to_dev, unstable_index_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1612_02557_amd import raduls
    assert torch.cuda.is_available()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    return raduls


def _as_void(a):
    a = np.ascontiguousarray(a)
    return a.view(np.dtype((np.void, a.shape[1]))).ravel()


def check(R, host, k, label):
    note(label)
    dev = to_dev(host)
    R.sort_inplace(dev, k, check=True)
    got = dev.cpu().numpy()
    want = oracle.sort(host, k)
    assert got.shape == want.shape
    bad = np.nonzero((got[:, :k] != want[:, :k]).any(axis=1))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} keys differ from the oracle's, first at {int(bad[0])}"
    assert np.array_equal(np.sort(_as_void(got)), np.sort(_as_void(host))), \
        f"{label}: output records are not a permutation of the input"


def spec(n, r=16, k=8, dist="uniform", payload="index", seed=41, **kw):
    return synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=dist, payload=payload, seed=seed, **kw)


# around the finishing capacity (17K records of 16 bytes), the one-workgroup
# bucket limit (2^20 records of 16 bytes) and several stripes
SIZES = [0, 1, 2, 3, 31, 33, 1000, 4097, 17408, 17409, 20000, 65537, 300_001, 1_048_576, 1_048_577,
         2_100_000, 5_000_003]


@pytest.mark.parametrize("n", SIZES)
def test_sizes(R, n):
    check(R, synth.generate(spec(n)), 8, f"inplace uniform r=16 k=8 n={n}")


@pytest.mark.parametrize("dist", ["zipf", "prefix", "bytes"])
@pytest.mark.parametrize("n", [70_001, 2_500_000])
def test_distributions(R, dist, n):
    check(R, synth.generate(spec(n, dist=dist, seed=42)), 8, f"inplace {dist} r=16 k=8 n={n}")


@pytest.mark.parametrize("r,k", [(4, 4), (8, 8), (12, 3), (16, 16), (20, 5), (24, 16), (32, 8), (64, 16), (60, 9),
                                 (8, 1), (12, 12)])
@pytest.mark.parametrize("n", [150_001, 2_200_000])
def test_record_shapes(R, r, k, n):
    host = synth.generate(spec(n, r=r, k=k, payload="random", seed=43))
    check(R, host, k, f"inplace r={r} k={k} n={n}")


def _keyed(keys, r=16):
    n = len(keys)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, :8] = np.asarray(keys, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("n", [50_000, 1_500_000])
def test_adversarial(R, n, rng):
    """All keys equal; two values; one digit shared by all keys (constant
    digit); keys already sorted and reversed; a heavy key among uniform ones;
    runs of equal keys the length of a block."""
    ar = np.arange(n, dtype=np.uint64)
    cases = {
        "all_equal": np.full(n, 7, dtype=np.uint64),
        "two_values": (ar % np.uint64(2)) * np.uint64(1 << 63),
        "shared_top_byte": np.uint64(0xAB << 56) | rng.integers(0, 1 << 56, n, dtype=np.uint64),
        "sorted": ar * np.uint64(12345),
        "reversed": (np.uint64(n) - ar) * np.uint64(12345),
        "heavy": np.where(rng.random(n) < 0.4, np.uint64(99), rng.integers(0, 1 << 64, n, dtype=np.uint64)),
        "block_runs": (ar // np.uint64(32)) * np.uint64(0x0101010101010101),
        "low_byte_only": ar % np.uint64(256),
    }
    for name, keys in cases.items():
        check(R, _keyed(keys.astype(np.uint64)), 8, f"inplace {name} n={n}")


@pytest.mark.parametrize("slb", [1, 3, 16, 64])
@pytest.mark.parametrize("dist", ["uniform", "zipf", "prefix"])
def test_many_stripes(R, monkeypatch, slb, dist):
    """Stripes of a few blocks (test-only setting read per call), so that a
    bucket of a few hundred thousand records has hundreds of stripes and its
    children's ranges cross many of them."""
    monkeypatch.setenv("RADULS_TEST_IP_SLB", str(slb))
    for n, r, k in [(200_003, 16, 8), (90_001, 8, 8), (120_000, 32, 16)]:
        check(R, synth.generate(spec(n, r=r, k=k, dist=dist, seed=44)), k,
              f"inplace slb={slb} {dist} r={r} k={k} n={n}")


def test_stripe_length_grows_with_n(R, monkeypatch):
    """A bucket has at most 8192 stripes: with stripes of one block asked
    for (test-only setting), 400,000 records of 16 bytes (12,500 blocks) get
    stripes of two blocks instead, and sort exactly."""
    monkeypatch.setenv("RADULS_TEST_IP_SLB", "1")
    check(R, synth.generate(spec(400_000, seed=47)), 8, "inplace slb=1 n=400000 (stripe length grows)")


def test_repeat_and_sizes_in_turn(R):
    """Calls of different sizes and shapes one after another (the workspace
    grows and is reused)."""
    for n, r, k in [(3_000_000, 16, 8), (1000, 16, 8), (400_000, 32, 16), (2_000_000, 8, 8), (5, 64, 16)]:
        check(R, synth.generate(spec(n, r=r, k=k, payload="random", seed=45)), k, f"inplace turn r={r} k={k} n={n}")


def test_full_size_sampled(R):
    """2^30 records of 16 bytes (8-byte uniform keys, payload = input index),
    the in-place benchmark's workload, checked on the device: every output
    record is the input record its payload names, every input index occurs,
    keys never decrease."""
    import torch
    from synth import device as sdev
    n = 1 << 30
    note(f"inplace full size n={n}")
    s = spec(n, seed=46)
    inp = sdev.generate(s)
    out = inp.clone()
    R.sort_inplace(out, 8, check=True)
    msg = unstable_index_check(out, inp, 8)
    assert msg is None, msg
    del inp, out
    torch.cuda.empty_cache()
