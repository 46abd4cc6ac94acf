"""Helpers shared by the GPU tests (no sorting arithmetic here)."""
import sys

import numpy as np


def note(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(host):
    import torch
    return torch.from_numpy(np.ascontiguousarray(host)).to("cuda")


def first_diff(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.nonzero((got != want).any(axis=1))[0]
    if len(bad) == 0:
        return "identical"
    i = int(bad[0])
    return f"{len(bad)} records differ, first at {i}: got {got[i].tolist()} want {want[i].tolist()}"


def _ukey(w):
    """Unsigned 64-bit order as signed order."""
    import torch
    return w ^ torch.iinfo(torch.int64).min


def _lex_less(a, b):
    """Elementwise a < b for lists of equal-length int64 columns, most significant first."""
    lt = a[-1] < b[-1]
    for x, y in zip(reversed(a[:-1]), reversed(b[:-1])):
        lt = (x < y) | ((x == y) & lt)
    return lt


def exact_index_check(out_dev, inp_dev, rec_bytes: int = 16, key_bytes: int = 8, chunk: int = 1 << 27):
    """Exactness test of a device sort, run on the device with torch ops.

    Records whose key is 8 or 16 bytes and whose next 8 bytes hold the input
    index (the generator's ``index`` payload): the output equals the stable
    sort of the input iff (i) every output record equals the input record its
    payload names and (ii) (key, payload) strictly increases along the output
    (then the payloads are distinct, the output is a permutation of the input,
    and the order is the unique stable order).  Checked ``chunk`` records at a
    time, so that the check of a 2^32-record sort fits next to its buffers.
    Key-only records (rec_bytes == key_bytes in {8, 16}): the output equals
    the input keys sorted by torch (two stable passes for 16-byte keys).
    Returns None (exact), a message, or "unchecked" for other formats.
    """
    import torch
    n = out_dev.shape[0]
    if n == 0:
        return None
    if key_bytes not in (8, 16) or rec_bytes % 8:
        return "unchecked"
    kw = key_bytes // 8
    if rec_bytes == key_bytes:
        # columns gathered one at a time, `chunk` indices per gather
        o = out_dev.view(torch.int64).view(n, kw)
        cols = [inp_dev.view(torch.int64).view(n, kw)[:, w].contiguous() for w in range(kw)]

        def gather(src, idx):
            out = torch.empty_like(src)
            for a in range(0, n, chunk):
                b = min(n, a + chunk)
                out[a:b] = src[idx[a:b]]
            return out

        perm = torch.sort(_ukey(cols[0]), stable=True).indices
        if kw == 2:
            hi = gather(_ukey(cols[1]), perm)
            perm = gather(perm, torch.sort(hi, stable=True).indices)
            del hi
        for w in range(kw):
            for a in range(0, n, chunk):
                b = min(n, a + chunk)
                if not torch.equal(cols[w][perm[a:b]], o[a:b, w]):
                    return f"output in [{a}, {b}) is not the sorted input"
        return None
    if rec_bytes < key_bytes + 8:
        return "unchecked"
    o = out_dev.view(torch.int64).view(n, -1)
    prev = None
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        idx = o[a:b, kw]
        if int(idx.min()) < 0 or int(idx.max()) >= n:
            return "payload out of range"
        if not torch.equal(inp_dev[idx], out_dev[a:b]):
            return f"an output record in [{a}, {b}) differs from the input record its payload names"
        cols = [_ukey(o[a:b, w]) for w in reversed(range(kw))] + [idx]   # most significant first
        if prev is not None:
            cols = [torch.cat([p, c]) for p, c in zip(prev, cols)]
        ok = _lex_less([c[:-1] for c in cols], [c[1:] for c in cols])
        if not bool(ok.all()):
            j = int(torch.nonzero(~ok)[0]) + a - (1 if prev is not None else 0)
            return f"order broken at {j}"
        prev = [c[-1:].clone() for c in cols]
        del cols, ok
    return None


def unstable_index_check(out_dev, inp_dev, key_bytes: int = 8, chunk: int = 1 << 27):
    """Exactness test of a device sort that need not be stable, on the device.

    Records whose key is 8 or 16 bytes followed by the input index (8 bytes):
    the output is a correct unstable sort of the input iff every output record
    equals the input record its payload names, every input index occurs
    (then the output is a permutation of the input), and the keys never
    decrease along the output.  Returns None (exact) or a message."""
    import torch
    n = out_dev.shape[0]
    if n == 0:
        return None
    kw = key_bytes // 8
    o = out_dev.view(torch.int64).view(n, -1)
    seen = torch.zeros(n, dtype=torch.bool, device=out_dev.device)
    prev = None
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        idx = o[a:b, kw]
        if int(idx.min()) < 0 or int(idx.max()) >= n:
            return "payload out of range"
        if not torch.equal(inp_dev[idx], out_dev[a:b]):
            return f"an output record in [{a}, {b}) differs from the input record its payload names"
        seen[idx] = True
        cols = [_ukey(o[a:b, w]) for w in reversed(range(kw))]   # most significant first
        if prev is not None:
            cols = [torch.cat([p, c]) for p, c in zip(prev, cols)]
        gt = _lex_less([c[1:] for c in cols], [c[:-1] for c in cols])   # next key below this one
        if bool(gt.any()):
            j = int(torch.nonzero(gt)[0]) + a - (1 if prev is not None else 0)
            return f"keys decrease at {j}"
        prev = [c[-1:].clone() for c in cols]
        del cols, gt
    if not bool(seen.all()):
        return "some input records are missing from the output"
    return None
