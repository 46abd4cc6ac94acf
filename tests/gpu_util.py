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


def exact_index_check(out_dev, inp_dev, key_bytes: int = 8):
    """Exactness test for 16-byte records with an 8-byte key and payload = index.

    The output equals the stable sort of the input iff (i) every output record
    equals the input record its payload names and (ii) (key, payload) strictly
    increases along the output (then the payloads are distinct, the output is
    a permutation of the input, and the order is the unique stable order).
    Runs on the device with torch ops; returns None or a message.
    """
    import torch
    n = out_dev.shape[0]
    if n == 0:
        return None
    o = out_dev.view(torch.int64).view(n, -1)
    key = o[:, 0]
    idx = o[:, 1]
    if int(idx.min()) < 0 or int(idx.max()) >= n:
        return "payload out of range"
    if not torch.equal(inp_dev[idx], out_dev):
        return "an output record differs from the input record its payload names"
    ks = key ^ torch.iinfo(torch.int64).min  # unsigned order as signed order
    a, b = ks[:-1], ks[1:]
    ok = (a < b) | ((a == b) & (idx[:-1] < idx[1:]))
    if not bool(ok.all()):
        j = int(torch.nonzero(~ok)[0])
        return f"order broken at {j}"
    return None
