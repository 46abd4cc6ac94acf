"""The committed scheduler network against the heuristic, offline.

``tests/fixtures/sched_holdout.npz`` holds sampled finishing jobs traced on
held-out workloads (new data, other seeds): each row has the job's nine
features, its feasible procedures, the measured time of every feasible
procedure and the heuristic's choice.  It is a measured evaluation set, not
a parity expectation.  The network is evaluated here by the float64/float32
oracle (``mlp_ref.forward_f32``), with the sorter's rules for taking its
answer (masked argmin, lowest procedure on ties, the heuristic's choice
outside the training range); the regret (``sched_ref.regret``) of its
choices must be below the heuristic's."""
import os
import struct

import numpy as np

from oracle import mlp_ref, sched_ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1612_02557_amd", "models", "sched_mlp.rdls")
FIXTURE = os.path.join(ROOT, "tests", "fixtures", "sched_holdout.npz")
F, H, P = 9, 32, 3
OOD_Z = 4.0


def load_blob(path):
    b = open(path, "rb").read()
    assert b[:8] == b"RDLSMLP1"
    assert struct.unpack("<3I", b[8:20]) == (F, H, P)
    a = np.frombuffer(b[20:-4], dtype="<f4")
    n = mlp_ref.n_params(F, H, P)
    assert a.size == n + 2 * F
    return a[:n], a[n:n + F], a[n + F:]


def learned_choices(theta, mean, scale, rows):
    X = (rows["features"].astype(np.float32) - mean) / scale
    Y = mlp_ref.forward_f32(theta, X, F, H, P)
    feas = rows["observed"].astype(np.int64)
    out = []
    for x, y, f, h in zip(X, Y, feas, rows["chosen"]):
        if np.abs(x).max() > OOD_Z:
            out.append(int(h))
            continue
        cand = [q for q in range(P) if (f >> q) & 1]
        out.append(min(cand, key=lambda q: (y[q], q)))
    return out


def times_of(rows):
    return [[float(t[q]) if (int(f) >> q) & 1 else None for q in range(P)]
            for t, f in zip(rows["ticks"], rows["observed"])]


def test_fixture_is_consistent():
    rows = np.load(FIXTURE)
    n = len(rows["chosen"])
    assert n >= 1000
    for f, c, t in zip(rows["observed"], rows["chosen"], rows["ticks"]):
        assert bin(int(f)).count("1") >= 2 and (int(f) >> int(c)) & 1
        assert all(t[q] > 0 for q in range(P) if (int(f) >> q) & 1)


def test_trained_network_beats_heuristic_on_held_out_jobs():
    theta, mean, scale = load_blob(MODEL)
    rows = np.load(FIXTURE)
    times = times_of(rows)
    heur = sched_ref.regret([int(c) for c in rows["chosen"]], times)
    learned = sched_ref.regret(learned_choices(theta, mean, scale, rows), times)
    print(f"held-out regret: heuristic {heur:.4f}, learned {learned:.4f}")
    assert learned < heur
