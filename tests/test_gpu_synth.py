"""The device generator writes exactly the bytes of the host generator.

Every benchmark, profile and training input is produced on the device by
``synth.device``; these cases pin it to ``synth.gen`` byte for byte, for each
key distribution, record and key size, payload kind, and a start index
i0 > 0 (chunked generation of large inputs starts there).
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dist", ["uniform", "zipf", "prefix", "mix", "bytes"])
@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (16, 16), (32, 8), (32, 16)])
@pytest.mark.parametrize("payload", ["index", "random"])
def test_device_generator_matches_host(dist, r, k, payload):
    import torch
    from synth import device
    if dist == "bytes":
        k = min(k, 5) if r > 8 else 5
    n, i0 = 3001, 123457
    note(f"synth dist={dist} r={r} k={k} payload={payload} i0={i0}")
    spec = synth.Spec(n=i0 + n, rec_bytes=r, key_bytes=k, dist=dist, payload=payload, seed=7)
    want = synth.generate(spec, i0, i0 + n)
    out = torch.empty((n, r), dtype=torch.uint8, device="cuda")
    device.fill(out, spec, i0=i0)
    got = out.cpu().numpy()
    assert np.array_equal(got, want), f"first differing record {int(np.argmax((got != want).any(axis=1)))}"


@pytest.mark.parametrize("r,k,bases", [(8, 8, 21), (8, 8, 32), (16, 8, 31), (16, 16, 40), (16, 16, 64),
                                      (32, 16, 55), (4, 4, 3)])
def test_device_kmers_match_host(r, k, bases):
    import torch
    from synth import device
    n, i0 = 5003, 77777
    note(f"synth kmer r={r} k={k} K={bases} i0={i0}")
    spec = synth.Spec(n=i0 + n, rec_bytes=r, key_bytes=k, dist="kmer", kmer_len=bases, payload="random", seed=9)
    want = synth.generate(spec, i0, i0 + n)
    out = torch.empty((n, r), dtype=torch.uint8, device="cuda")
    device.fill(out, spec, i0=i0)
    got = out.cpu().numpy()
    assert np.array_equal(got, want), f"first differing record {int(np.argmax((got != want).any(axis=1)))}"


def test_device_segments_match_host():
    import torch
    from synth import device
    note("synth segments")
    spec = synth.Spec(n=0, rec_bytes=16, key_bytes=8, dist="uniform", payload="index", seed=4)
    sizes = np.array([5, 0, 1000, 1, 77, 2048], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    dists = np.array([0, 1, 1, 0, 1, 0])
    got = device.generate_segments(spec, off, dists).cpu().numpy()
    want = synth.gen.generate_segments(spec, off, dists)
    assert np.array_equal(got, want)
