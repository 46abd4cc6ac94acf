"""The entry point that allocates nothing (raduls_sort_noalloc) against the
allocating raduls_sort, byte for byte, through the C ABI.  Collected last:
the fixed scratch array is shared by every call on the GPU, so these tests
also see whatever earlier calls left in it."""
import numpy as np
import pytest

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


def both(R, host, k):
    """(output of raduls_sort, output of raduls_sort_noalloc) on the same input."""
    import torch
    a = to_dev(host)
    R.sort(a, k, check=True)
    b = to_dev(host)
    tmp = torch.empty_like(b)
    R.sort_noalloc(b, k, tmp, check=True)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("first,second", [((2_000_003, 16, 8, "mix"), (70_001, 16, 8, "uniform")),
                                          ((1_000_000, 32, 16, "zipf"), (4097, 8, 8, "prefix"))])
def test_two_calls_in_a_row_match_the_allocating_sort(R, first, second):
    for n, r, k, dist in (first, second):
        note(f"noalloc n={n} r={r} k={k} {dist}")
        host = synth.generate(synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=dist, payload="random", seed=11))
        want, got = both(R, host, k)
        assert np.array_equal(got, want), f"n={n} r={r} k={k} {dist}: {first_diff(got, want)}"


def test_many_small_calls_reuse_the_scratch(R):
    import torch
    rng = np.random.default_rng(7)
    for i in range(40):
        n = int(rng.integers(2, 50_000))
        note(f"noalloc repeat {i} n={n}")
        host = synth.generate(synth.Spec(n=n, rec_bytes=16, key_bytes=8, dist="zipf", seed=100 + i))
        want, got = both(R, host, 8)
        assert np.array_equal(got, want), f"call {i} n={n}: {first_diff(got, want)}"
    torch.cuda.synchronize()


def test_too_large_for_the_scratch_is_refused_before_device_work(R):
    import torch
    n = 1 << 23  # workspace above 64 MiB at 64-byte records
    assert R.lib().raduls_workspace_bytes(n, 64, 16) > R.NOALLOC_SCRATCH_BYTES
    rec = torch.zeros((n, 64), dtype=torch.uint8, device="cuda")
    rec[:, 0] = 1
    tmp = torch.empty_like(rec)
    with pytest.raises(R.RadulsError) as e:
        R.sort_noalloc(rec, 16, tmp)
    assert e.value.code == R.EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((rec[:, 0] == 1).all()) and bool((rec[:, 1:] == 0).all())
