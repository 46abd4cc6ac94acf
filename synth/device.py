"""Device generator: fills CUDA tensors with exactly the bytes of ``synth.gen``."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import gen

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libsynth.so")
_lib = None
_cdf_cache = {}


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "csrc", "synth_gen.hip")
    cmd = ["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", SO + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    os.replace(SO + ".tmp", SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is not built")
        import torch  # noqa: F401  (bind to the HIP runtime PyTorch loads)
        L = ctypes.CDLL(SO)
        v = ctypes.c_void_p
        L.synth_fill.argtypes = [v, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                 ctypes.c_int, v, v, ctypes.c_uint32, v]
        L.synth_fill.restype = ctypes.c_int
        _lib = L
    return _lib


def _bases(spec: gen.Spec) -> np.ndarray:
    seed = spec.seed
    S = gen.STREAMS
    b = [gen.stream_base(seed, S["KEY"]), gen.stream_base(seed, S["KEY_HI"]), gen.stream_base(seed, S["ZIPF"]),
         gen.stream_base(seed, S["MIX"]), gen.stream_base(seed, S["ZIPF_SALT_LO"]),
         gen.stream_base(seed, S["ZIPF_SALT_HI"])]
    b += [gen.stream_base(seed, S["PAYLOAD"] + w) for w in range(16)]
    b += [gen.stream_base(seed, S["PREFIX"]) >> 40]
    b += [gen.stream_base(seed, S["GENOME"]), gen.stream_base(seed, S["KMERPOS"]), gen.stream_base(seed, S["KMERERR"])]
    b += [spec.windows, spec.bases]
    return np.array(b, dtype=np.uint64)


def _cdf(s: float, m: int, device):
    import torch
    key = (s, m, str(device))
    if key not in _cdf_cache:
        _cdf_cache[key] = torch.from_numpy(gen.zipf_cdf(s, m)).to(device)
    return _cdf_cache[key]


def fill(out, spec: gen.Spec, i0: int = 0, dist: str | None = None, stream=None):
    """Write records i0 .. i0+len(out)-1 of ``spec`` into ``out`` (CUDA uint8 [m, rec_bytes])."""
    import torch
    d = dist or spec.dist
    code = gen.DIST_CODE[d]
    cdf = _cdf(spec.zipf_s, spec.zipf_m, out.device)
    bases = _bases(spec)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = lib().synth_fill(out.data_ptr(), i0, out.shape[0], spec.rec_bytes, spec.key_bytes, code,
                          1 if spec.payload == "index" else 0, bases.ctypes.data, cdf.data_ptr(), spec.zipf_m, st)
    if rc:
        raise RuntimeError(f"synth_fill failed ({rc})")
    return out


def generate(spec: gen.Spec, device="cuda"):
    import torch
    out = torch.empty((spec.n, spec.rec_bytes), dtype=torch.uint8, device=device)
    return fill(out, spec)


def generate_segments(spec: gen.Spec, off: np.ndarray, dists: np.ndarray, device="cuda", out=None, segs=None):
    """All records of a batch (segment s with key distribution dists[s]); global index payload.

    With ``out`` the records are written there; with ``segs = (s0, s1)`` only
    segments s0 .. s1-1 are written (at their global positions in ``out``).
    """
    import torch
    n = int(off[-1])
    if out is None:
        out = torch.empty((n, spec.rec_bytes), dtype=torch.uint8, device=device)
    # consecutive segments of one distribution are filled by one launch
    s, S = (0, len(dists)) if segs is None else segs
    while s < S:
        e = s
        while e + 1 < S and dists[e + 1] == dists[s]:
            e += 1
        a, b = int(off[s]), int(off[e + 1])
        if b > a:
            fill(out[a:b], spec, i0=a, dist="zipf" if dists[s] == 1 else "uniform")
        s = e + 1
    return out
