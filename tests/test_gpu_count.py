"""GPU parity of duplicate removal with counts (k-mer counting, paper Sec. 5):
``raduls_count_runs`` and ``raduls_sort_count`` against the oracle, byte for
byte (unique records) and exactly (counts)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1612_02557_amd import raduls
    assert torch.cuda.is_available()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    return raduls


def check_runs(R, sorted_host, k, label, in_place=False):
    note(label)
    dev = to_dev(sorted_host)
    u, c = R.count_runs(dev, k, uniq=dev if in_place else None, check=True)
    wu, wc = oracle.count_runs(sorted_host, k)
    got_u, got_c = u.cpu().numpy(), c.cpu().numpy().astype(np.uint64)
    assert got_u.shape == wu.shape, f"{label}: {len(got_u)} runs, want {len(wu)}"
    assert np.array_equal(got_u, wu), f"{label}: unique records differ"
    assert np.array_equal(got_c, wc), f"{label}: counts differ at {int(np.argmax(got_c != wc))}"


SIZES = [1, 2, 31, 64, 255, 2047, 2048, 2049, 4095, 4096, 4097, 8193, 100_000, 1_000_003]


@pytest.mark.parametrize("n", SIZES)
def test_kmers_16_16(R, n):
    host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=16, dist="kmer", payload="index", seed=31))
    check_runs(R, oracle.sort(host, 16), 16, f"kmer r=16 k=16 n={n}")


@pytest.mark.parametrize("r,k", [(4, 4), (8, 8), (12, 3), (16, 8), (20, 5), (24, 16), (32, 16), (64, 16), (60, 9)])
@pytest.mark.parametrize("n", [777, 70_001])
def test_record_shapes(R, r, k, n):
    if k >= 2:
        spec = synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist="kmer", kmer_len=min(4 * k, 64), kmer_cov=5,
                          payload="random", seed=32)
    else:
        spec = synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist="bytes", payload="random", seed=32)
    host = synth.generate(spec)
    check_runs(R, oracle.sort(host, k), k, f"kmer r={r} k={k} n={n}")


def _keyed(keys, r=16):
    n = len(keys)
    rec = np.zeros((n, r), dtype=np.uint8)
    rec[:, :8] = np.asarray(keys, dtype="<u8").view(np.uint8).reshape(n, 8)
    rec[:, 8:16] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    return rec


@pytest.mark.parametrize("n", [5000, 300_000])
def test_run_structures(R, n, rng):
    """Runs that span many tiles, end exactly on tile boundaries, or are all
    of length one; a single key throughout."""
    tile = 4096  # records per tile of 16-byte records
    cases = {
        "all_equal": np.full(n, 42, dtype=np.uint64),
        "all_distinct": np.arange(n, dtype=np.uint64) * np.uint64(977),
        "tile_runs": np.arange(n, dtype=np.uint64) // np.uint64(tile),
        "tile_runs_shifted": (np.arange(n, dtype=np.uint64) + np.uint64(1)) // np.uint64(tile),
        "half_tile_runs": np.arange(n, dtype=np.uint64) // np.uint64(tile // 2),
        "long_runs": np.sort(rng.integers(0, 7, n, dtype=np.uint64)),
        "pairs": np.arange(n, dtype=np.uint64) // np.uint64(2),
        "zipf": None,
    }
    for name, keys in cases.items():
        if keys is None:
            host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=8, dist="zipf", seed=33))
            check_runs(R, oracle.sort(host, 8), 8, f"runs {name} n={n}")
        else:
            check_runs(R, _keyed(keys), 8, f"runs {name} n={n}")


@pytest.mark.parametrize("n", [3000, 500_000])
def test_in_place(R, n):
    host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=16, dist="kmer", kmer_cov=3, seed=34))
    check_runs(R, oracle.sort(host, 16), 16, f"in place n={n}", in_place=True)


@pytest.mark.parametrize("where", ["new", "tmp", "records"])
def test_sort_count(R, where):
    import torch
    n = 1_500_000
    note(f"sort_count uniq={where} n={n}")
    host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=16, dist="kmer", seed=35))
    dev = to_dev(host)
    tmp = torch.empty_like(dev)
    uniq = {"new": None, "tmp": tmp, "records": dev}[where]
    u, c = R.sort_count(dev, 16, tmp=tmp, uniq=uniq, check=True)
    wu, wc = oracle.sort_count(host, 16)
    assert np.array_equal(u.cpu().numpy(), wu)
    assert np.array_equal(c.cpu().numpy().astype(np.uint64), wc)
    if where != "records":
        assert np.array_equal(dev.cpu().numpy(), oracle.sort(host, 16)), "records keep the sorted order"


def test_empty(R):
    import torch
    note("count_runs n=0")
    dev = torch.zeros((0, 16), dtype=torch.uint8, device="cuda")
    u, c = R.count_runs(dev, 8, check=True)
    assert u.shape[0] == 0 and c.shape[0] == 0


def test_sort_count_full_size_sampled(R):
    """2^27 16-byte k-mers (16-byte keys), sorted and counted on the device;
    checked by properties that hold at any size (counts sum to n, unique keys
    strictly increase, every unique record is the record that starts its run
    in the sorted array) and, for sampled runs, against the oracle's count
    of that key over the input."""
    import torch
    from synth import device as sdev
    n = 1 << 27
    note(f"sort_count full size n={n}")
    spec = synth.Spec(n=n, rec_bytes=16, key_bytes=16, dist="kmer", payload="index", seed=36)
    dev = sdev.generate(spec)
    tmp = torch.empty_like(dev)
    u, c = R.sort_count(dev, 16, tmp=tmp, uniq=tmp, check=True)
    U = u.shape[0]
    assert int(c.sum().item()) == n
    assert int(c.min().item()) >= 1
    w = u.view(torch.int64).view(U, 2)
    hi, lo = w[:, 1] ^ torch.iinfo(torch.int64).min, w[:, 0] ^ torch.iinfo(torch.int64).min
    inc = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))
    assert bool(inc.all().item()), "unique keys strictly increase"
    starts = torch.cumsum(c, 0) - c
    assert torch.equal(u, dev[starts]), "each unique record starts its run in the sorted array"
    # sampled keys: count over the input generated on the host in chunks
    rng = np.random.default_rng(7)
    pick = rng.integers(0, U, 64)
    uw = w[torch.from_numpy(pick).to("cuda")].cpu().numpy().view(np.uint64)   # (64, 2): lo, hi words
    cw = c[torch.from_numpy(pick).to("cuda")].cpu().numpy()
    want = {(int(a), int(b)): int(x) for (a, b), x in zip(uw, cw)}
    seen = dict.fromkeys(want, 0)
    step = 1 << 24
    for a in range(0, n, step):
        part = synth.generate(spec, a, min(n, a + step))
        kw = np.ascontiguousarray(part[:, :16]).view("<u8")
        hit = np.nonzero(np.isin(kw[:, 0], uw[:, 0]))[0]
        for i in hit:
            key = (int(kw[i, 0]), int(kw[i, 1]))
            if key in seen:
                seen[key] += 1
    assert seen == want


def test_wait_limit_reported(R, monkeypatch):
    """A look-back wait limit of 0 (test-only, read from the environment per
    call) makes every tile after the first give up at once; the kernel still
    exits and check=True reports EDEVICE; the next call is exact."""
    note("count_runs wait limit 0 -> EDEVICE")
    host = synth.generate(synth.Spec(n=200_000, rec_bytes=16, key_bytes=16, dist="kmer", seed=37))
    sh = oracle.sort(host, 16)
    dev = to_dev(sh)
    monkeypatch.setenv("RADULS_TEST_SPIN_LIMIT", "0")
    with pytest.raises(R.RadulsError) as e:
        R.count_runs(dev, 16, check=True)
    assert e.value.code == R.EDEVICE
    monkeypatch.delenv("RADULS_TEST_SPIN_LIMIT")
    check_runs(R, sh, 16, "after the wait-limit case")
