"""Host (numpy) generator of seeded synthetic records.

Random source: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  ``mix64`` is its output
function, a bijection of 64-bit words; the i-th value of a stream is
``mix64(base + (i + 1) * GAMMA)``, i.e. the i-th output of SplitMix64 started
from state ``base(seed, stream)``.  Everything below is a pure function of
(seed, stream, index), so any index range regenerates on its own and the
device generator (``synth.device``) reproduces it byte for byte.

Record bytes for record i (key_bytes = k, rec_bytes = r):
  * key = bytes [0, k), an unsigned little-endian integer:
      uniform : bytes 0..7 from stream KEY, bytes 8..15 from stream KEY_HI
      zipf    : rank j in [1, m] with P(j) proportional to j**-s (inverse-CDF
                draw from stream ZIPF); key words mix64(j ^ salt_lo) and
                mix64(j ^ salt_hi), so the m ranks give m distinct keys
      prefix  : uniform key whose top 24 bits are replaced by a per-seed
                constant P24 (requires k in {8, 16})
      mix     : per record, from stream MIX: uniform with probability 1/2,
                zipf with 3/10, prefix with 1/5
      bytes   : same as uniform (every key byte random); any k
      kmer    : k-mers of reads drawn from one synthetic genome (the data of
                the k-mer counting application, paper Sec. 4-5): a genome of
                W + K - 1 bases, two bits each, 32 bases per word of stream
                GENOME; W = max(n // kmer_cov, 1) start positions; record i
                takes the K bases at position p = (stream KMERPOS) mod W,
                i.e. bits [2p, 2p + 2K) of the genome, and with probability
                1/64 (top 6 bits of stream KMERERR zero) one base
                substituted: base (e & 0xFFFF) mod K XOR ((e >> 16) mod 3 + 1)
                (a sequencing error).  Every genome position is drawn about
                kmer_cov times, so most keys repeat.  K = kmer_len, at most
                4 * key_bytes
  * payload = bytes [k, r):
      index   : the first 8 payload bytes hold i as a little-endian uint64
                (truncated if fewer), later bytes random
      random  : every payload byte random
    payload byte p (0-based, from byte k) that is random is byte (p % 8) of
    stream PAYLOAD + p // 8.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

STREAMS = {
    "KEY": 1,
    "KEY_HI": 2,
    "ZIPF": 8,
    "MIX": 9,
    "SEGSIZE": 10,
    "SEGDIST": 11,
    "ZIPF_SALT_LO": 12,
    "ZIPF_SALT_HI": 13,
    "PREFIX": 14,
    "GENOME": 15,
    "KMERPOS": 16,
    "KMERERR": 17,
    "PAYLOAD": 32,  # 32, 33, ... one stream per 8 payload bytes
}

# mixture thresholds on the top 53 bits of the MIX stream value
MIX_T_UNIFORM = 1 << 52                 # 1/2 of 2**53
MIX_T_ZIPF = 7205759403792793           # floor(0.8 * 2**53)

DISTS = ("uniform", "zipf", "prefix", "mix", "bytes", "kmer")
DIST_CODE = {"uniform": 0, "zipf": 1, "prefix": 2, "mix": 3, "bytes": 0, "kmer": 4}


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def splitmix64(x: int) -> int:
    """SplitMix64 output function on a Python int (mod 2**64)."""
    z = x & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def stream_base(seed: int, stream: int) -> int:
    return splitmix64(splitmix64(seed & M64) ^ ((stream * GAMMA) & M64))


def uniform_u64(seed: int, stream: int, i0: int, i1: int) -> np.ndarray:
    """Values i0..i1-1 of a stream as uint64."""
    base = np.uint64(stream_base(seed, stream))
    idx = np.arange(i0, i1, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        state = base + idx * np.uint64(GAMMA)
    return _mix64_np(state)


def zipf_cdf(s: float = 1.1, m: int = 1 << 20) -> np.ndarray:
    """Cumulative probabilities of ranks 1..m, P(j) proportional to j**-s.

    Sequential cumulative sum in float64 (np.cumsum), normalised by its last
    element; the device generator uses this same array.
    """
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_ranks(u: np.ndarray, cdf: np.ndarray) -> np.ndarray:
    """Rank j (1-based) = 1 + number of cdf entries <= x, x = top 53 bits / 2**53."""
    x = (u >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    idx = np.searchsorted(cdf, x, side="right")
    idx = np.minimum(idx, len(cdf) - 1)
    return idx.astype(np.uint64) + np.uint64(1)


@dataclasses.dataclass(frozen=True)
class Spec:
    n: int
    rec_bytes: int = 16
    key_bytes: int = 8
    dist: str = "uniform"
    payload: str = "index"
    seed: int = 1
    zipf_s: float = 1.1
    zipf_m: int = 1 << 20
    kmer_len: int = 0        # bases per k-mer (0: 4 * key_bytes)
    kmer_cov: int = 16       # records per genome position, on average

    def __post_init__(self):
        if self.dist not in DISTS:
            raise ValueError(f"unknown dist {self.dist}")
        if self.payload not in ("index", "random"):
            raise ValueError(f"unknown payload {self.payload}")
        if not (1 <= self.key_bytes <= 16 and self.key_bytes <= self.rec_bytes):
            raise ValueError("need 1 <= key_bytes <= min(rec_bytes, 16)")
        if self.dist in ("prefix", "mix") and self.key_bytes not in (8, 16):
            raise ValueError("prefix keys need key_bytes 8 or 16")
        if self.rec_bytes % 4 or self.rec_bytes > 64:
            raise ValueError("rec_bytes must be a multiple of 4, at most 64")
        if self.dist == "kmer" and not (1 <= self.bases <= 4 * self.key_bytes and self.kmer_cov >= 1):
            raise ValueError("kmer keys need 1 <= kmer_len <= 4 * key_bytes and kmer_cov >= 1")

    @property
    def bases(self) -> int:
        return self.kmer_len or 4 * self.key_bytes

    @property
    def windows(self) -> int:
        return max(self.n // self.kmer_cov, 1)


def _key_words(spec: Spec, i0: int, i1: int, dist_code: np.ndarray | None = None):
    """(lo, hi) uint64 words of the keys of records i0..i1-1."""
    seed = spec.seed
    lo = uniform_u64(seed, STREAMS["KEY"], i0, i1)
    hi = uniform_u64(seed, STREAMS["KEY_HI"], i0, i1)
    d = spec.dist
    if d in ("uniform", "bytes"):
        return lo, hi
    if d == "kmer":
        return _kmer_words(spec, i0, i1)
    if d == "mix":
        c = uniform_u64(seed, STREAMS["MIX"], i0, i1) >> np.uint64(11)
        code = np.where(c < np.uint64(MIX_T_UNIFORM), 0,
                        np.where(c < np.uint64(MIX_T_ZIPF), 1, 2)).astype(np.int8)
    elif dist_code is not None:
        code = dist_code
    else:
        code = np.full(i1 - i0, DIST_CODE[d], dtype=np.int8)
    zs = code == 1
    if zs.any():
        cdf = zipf_cdf(spec.zipf_s, spec.zipf_m)
        u = uniform_u64(seed, STREAMS["ZIPF"], i0, i1)[zs]
        j = zipf_ranks(u, cdf)
        slo = np.uint64(stream_base(seed, STREAMS["ZIPF_SALT_LO"]))
        shi = np.uint64(stream_base(seed, STREAMS["ZIPF_SALT_HI"]))
        lo[zs] = _mix64_np(j ^ slo)
        hi[zs] = _mix64_np(j ^ shi)
    ps = code == 2
    if ps.any():
        p24 = np.uint64(stream_base(seed, STREAMS["PREFIX"]) >> 40)
        mask40 = np.uint64((1 << 40) - 1)
        if spec.key_bytes == 8:
            lo[ps] = (p24 << np.uint64(40)) | (lo[ps] & mask40)
        else:
            hi[ps] = (p24 << np.uint64(40)) | (hi[ps] & mask40)
    return lo, hi


def _stream_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Values of a stream at arbitrary indices (uint64 array)."""
    base = np.uint64(stream_base(seed, stream))
    with np.errstate(over="ignore"):
        state = base + (idx.astype(np.uint64) + np.uint64(1)) * np.uint64(GAMMA)
    return _mix64_np(state)


def _kmer_words(spec: Spec, i0: int, i1: int):
    seed, K = spec.seed, spec.bases
    p = uniform_u64(seed, STREAMS["KMERPOS"], i0, i1) % np.uint64(spec.windows)
    b = p * np.uint64(2)
    w0 = b >> np.uint64(6)
    s = b & np.uint64(63)
    g0 = _stream_at(seed, STREAMS["GENOME"], w0)
    g1 = _stream_at(seed, STREAMS["GENOME"], w0 + np.uint64(1))
    g2 = _stream_at(seed, STREAMS["GENOME"], w0 + np.uint64(2))
    z = s == 0
    inv = np.where(z, np.uint64(1), np.uint64(64) - s)   # any shift where s == 0
    lo = np.where(z, g0, (g0 >> s) | (g1 << inv))
    hi = np.where(z, g1, (g1 >> s) | (g2 << inv))
    if 2 * K <= 64:
        hi = np.zeros_like(hi)
        if 2 * K < 64:
            lo &= np.uint64((1 << (2 * K)) - 1)
    elif 2 * K < 128:
        hi &= np.uint64((1 << (2 * K - 64)) - 1)
    e = uniform_u64(seed, STREAMS["KMERERR"], i0, i1)
    err = (e >> np.uint64(58)) == 0
    q = (e & np.uint64(0xFFFF)) % np.uint64(K)
    flip = ((e >> np.uint64(16)) % np.uint64(3)) + np.uint64(1)
    sh = (np.uint64(2) * q) & np.uint64(63)
    in_lo = err & (q < 32)
    in_hi = err & (q >= 32)
    lo = np.where(in_lo, lo ^ (flip << sh), lo)
    hi = np.where(in_hi, hi ^ (flip << sh), hi)
    return lo, hi


def generate(spec: Spec, i0: int = 0, i1: int | None = None,
             dist_code: np.ndarray | None = None) -> np.ndarray:
    """Records i0..i1-1 of ``spec`` as a uint8 array of shape (i1-i0, rec_bytes)."""
    if i1 is None:
        i1 = spec.n
    m = i1 - i0
    r, k = spec.rec_bytes, spec.key_bytes
    out = np.empty((m, r), dtype=np.uint8)
    lo, hi = _key_words(spec, i0, i1, dist_code)
    kb = np.empty((m, 16), dtype=np.uint8)
    kb[:, :8] = lo.astype("<u8").view(np.uint8).reshape(m, 8)
    kb[:, 8:] = hi.astype("<u8").view(np.uint8).reshape(m, 8)
    out[:, :k] = kb[:, :k]
    pl = r - k
    if pl > 0:
        nw = (pl + 7) // 8
        pw = np.empty((m, nw * 8), dtype=np.uint8)
        for w in range(nw):
            if w == 0 and spec.payload == "index":
                v = np.arange(i0, i1, dtype=np.uint64)
            else:
                v = uniform_u64(spec.seed, STREAMS["PAYLOAD"] + w, i0, i1)
            pw[:, 8 * w:8 * w + 8] = v.astype("<u8").view(np.uint8).reshape(m, 8)
        out[:, k:] = pw[:, :pl]
    return out


def segment_sizes(S: int, seed: int, lo: int = 1 << 10, hi: int = 1 << 22) -> np.ndarray:
    """m_s = floor(exp(U)), U uniform in [ln lo, ln hi): log-uniform sizes."""
    u = uniform_u64(seed, STREAMS["SEGSIZE"], 0, S) >> np.uint64(11)
    x = u.astype(np.float64) * (1.0 / (1 << 53))
    a, b = math.log(lo), math.log(hi)
    return np.floor(np.exp(a + x * (b - a))).astype(np.uint64)


def segment_offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    return off


def segment_dists(S: int, seed: int) -> np.ndarray:
    """Per segment: 0 = uniform keys, 1 = zipf keys (probability 1/2 each)."""
    u = uniform_u64(seed, STREAMS["SEGDIST"], 0, S)
    return (u >> np.uint64(63)).astype(np.int8)


def generate_segments(spec: Spec, off: np.ndarray, dists: np.ndarray) -> np.ndarray:
    """All records of a batch: segment s uses dist dists[s]; payload index is global."""
    n = int(off[-1])
    code = np.repeat(dists.astype(np.int8), np.diff(off).astype(np.int64))
    sp = dataclasses.replace(spec, n=n, dist="zipf")
    return generate(sp, 0, n, dist_code=code)
