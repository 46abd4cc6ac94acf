"""Generator determinism and distribution checks (host side)."""
import math

import numpy as np
import pytest

import synth


def test_splitmix64_published_vectors():
    # SplitMix64 started from state 0: first three outputs
    g = 0x9E3779B97F4A7C15
    assert synth.splitmix64(g) == 0xE220A8397B1DCDAF
    assert synth.splitmix64(2 * g) == 0x6E789E6AA1B965F4
    assert synth.splitmix64(3 * g) == 0x06C45D188009454F


@pytest.mark.parametrize("dist", ["uniform", "zipf", "prefix", "mix", "bytes", "kmer"])
def test_chunks_reproduce_slices(dist):
    k = 8 if dist != "bytes" else 5
    sp = synth.Spec(n=5000, rec_bytes=32, key_bytes=k, dist=dist, payload="random", seed=9)
    full = synth.generate(sp)
    np.testing.assert_array_equal(synth.generate(sp, 1234, 4321), full[1234:4321])
    np.testing.assert_array_equal(synth.generate(sp), full)


def test_index_payload():
    sp = synth.Spec(n=1000, rec_bytes=16, key_bytes=8, seed=1)
    a = synth.generate(sp)
    np.testing.assert_array_equal(a[:, 8:].copy().view("<u8").ravel(), np.arange(1000))


def test_zipf_top_frequency():
    n = 1 << 22
    a = synth.generate(synth.Spec(n=n, dist="zipf", seed=3))
    keys = a[:, :8].copy().view("<u8").ravel()
    _, c = np.unique(keys, return_counts=True)
    H = math.fsum(j ** -1.1 for j in range(1, (1 << 20) + 1))
    p1 = 1.0 / H
    assert abs(p1 - 0.1237) < 5e-4
    assert abs(c.max() / n - p1) < 5 * math.sqrt(p1 * (1 - p1) / n)


def test_zipf_keys_distinct_per_rank():
    cdf = synth.zipf_cdf(1.1, 1 << 12)
    assert cdf[-1] == 1.0 and np.all(np.diff(cdf) > 0)


def test_prefix_shared_bits():
    a = synth.generate(synth.Spec(n=4096, dist="prefix", seed=5))
    keys = a[:, :8].copy().view("<u8").ravel()
    assert len(np.unique(keys >> np.uint64(40))) == 1
    assert len(np.unique(keys & np.uint64((1 << 40) - 1))) > 4000


def test_mix_fractions():
    n = 1 << 18
    c = synth.uniform_u64(5, synth.STREAMS["MIX"], 0, n) >> np.uint64(11)
    fu = (c < np.uint64(synth.gen.MIX_T_UNIFORM)).mean()
    fz = ((c >= np.uint64(synth.gen.MIX_T_UNIFORM)) & (c < np.uint64(synth.gen.MIX_T_ZIPF))).mean()
    assert abs(fu - 0.5) < 0.01 and abs(fz - 0.3) < 0.01


def test_segment_sizes_log_uniform():
    s = synth.segment_sizes(10000, 4)
    assert s.min() >= 1024 and s.max() < (1 << 22)
    assert abs(np.log2(np.median(s)) - 16) < 0.2
    off = synth.segment_offsets(s)
    assert off[0] == 0 and off[-1] == s.sum()


@pytest.mark.parametrize("k,bases", [(8, 21), (8, 32), (16, 40), (16, 64)])
def test_kmers_are_genome_substrings(k, bases):
    """Error-free k-mer keys are K consecutive bases of one genome, read here
    base by base from Python integers (not the generator's word shifts);
    about 1/64 of the records carry exactly one substituted base."""
    n = 4000
    sp = synth.Spec(n=n, rec_bytes=16, key_bytes=k, dist="kmer", kmer_len=bases, kmer_cov=4, seed=5)
    rec = synth.generate(sp)
    S = synth.STREAMS
    pos = synth.uniform_u64(5, S["KMERPOS"], 0, n) % np.uint64(sp.windows)
    words = synth.uniform_u64(5, S["GENOME"], 0, (sp.windows + bases) // 32 + 2)
    genome = [int(w) for w in words]

    def base(q):
        return (genome[q // 32] >> (2 * (q % 32))) & 3

    errors = 0
    for i in range(n):
        key = int.from_bytes(bytes(rec[i, :k]), "little")
        want = sum(base(int(pos[i]) + j) << (2 * j) for j in range(bases))
        diff = key ^ want
        if diff:
            errors += 1
            j = (diff.bit_length() - 1) // 2
            assert diff >> (2 * j) in (1, 2, 3) and diff & ((1 << (2 * j)) - 1) == 0, "one base differs"
            assert j < bases
    assert abs(errors / n - 1 / 64) < 0.01
    # every start position is drawn about kmer_cov times
    assert abs(n / len(np.unique(pos)) - 4 / (1 - math.exp(-4))) < 0.3
