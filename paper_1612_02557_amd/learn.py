"""Learned per-bucket scheduler: traces, training, model blob, evaluation.

The paper sets the thresholds that pick a bin's procedure by hand
(Sec. 3.2-3.5).  Here a small network predicts, per finishing job, the
log-time of each procedure (RADIX, LSD, BITONIC) from nine features of the
bucket, and the sorter takes the cheapest feasible one:

1. ``collect``: sort seeded synthetic workloads with tracing on; sampled
   jobs run every feasible procedure (after one untimed warm-up run) and
   record each one's time, the others record the time of the procedure that
   ran.  Rows come from the library (64 bytes each).
2. ``train``: masked least squares on log2(ticks) of the sampled rows (at
   most a fixed number per workload), by the library's own
   kernels (``raduls_mlp_loss_grad``, ``raduls_mlp_adam``); this module only
   batches tensors.
3. ``regret`` on held-out sampled rows for the learned choice and for the
   heuristic that was running: sum(t(chosen) - min t) / sum(min t).
4. ``compare``: end-to-end time of whole sorts, heuristic vs learned.

``python -m paper_1612_02557_amd.learn --out DIR`` runs all four on the
current GPU and writes ``DIR/sched_mlp.rdls`` (the blob ``raduls_load_model``
takes), ``DIR/learn_report.json`` and ``DIR/sched_holdout.npz`` (a subset of
the held-out sampled rows, for an offline regret check).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import raduls

F, H, P = raduls.MLP_F, raduls.MLP_H, raduls.MLP_P
ROW = np.dtype([("features", "<f4", (9,)), ("chosen", "<u4"), ("count", "<u4"), ("observed", "<u4"),
                ("ticks", "<u4", (3,)), ("flags", "<u4")])
OOD_Z = 4.0  # RADULS_MLP_OOD_Z
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "sched_mlp.rdls")

# (log2 n, rec_bytes, key_bytes, distribution) of the training workloads:
# every size class from 2^22 to 2^30 (each gives a different job structure:
# queued buckets, one-workgroup passes, runs of small children) for each key
# distribution, 2^31 and 2^32 records of mixed keys, and other record
# shapes.  Held out: new data (other seeds) of the same shapes.
DISTS = ("uniform", "zipf", "prefix", "mix")
TRAIN = [(lg, 16, 8, d) for lg in range(22, 31) for d in DISTS] + \
        [(31, 16, 8, "mix"), (32, 16, 8, "mix")] + \
        [(lg, r, k, d) for lg in (23, 25, 28) for (r, k) in ((8, 8), (32, 8), (32, 16)) for d in ("uniform", "zipf", "prefix")]
HOLDOUT = [(lg, 16, 8, d) for lg in (23, 25, 27, 29) for d in DISTS] + \
          [(24, 32, 16, "zipf"), (24, 8, 8, "mix"), (29, 32, 16, "uniform"), (29, 8, 8, "prefix")]


def log(msg):
    print(f"[learn] {msg}", file=sys.stderr, flush=True)


def _inputs(lg, r, k, dist, seed):
    import synth
    from synth import device as sdev
    return sdev.generate(synth.Spec(n=1 << lg, rec_bytes=r, key_bytes=k, dist=dist, payload="index", seed=seed))


def collect(workloads, sample_period=3, seed=100, cap=1 << 21, per_workload=None):
    """Trace rows (numpy structured array) of sorting each workload once."""
    import torch
    out = []
    rows = torch.zeros(cap * ROW.itemsize, dtype=torch.uint8, device="cuda")
    for i, (lg, r, k, dist) in enumerate(workloads):
        data = _inputs(lg, r, k, dist, seed + i)
        tmp = torch.empty_like(data)
        raduls.set_trace(rows, sample_period)
        raduls.sort(data, k, tmp)
        cnt = raduls.trace_count()
        raduls.set_trace(None)
        raduls.sync_check()
        tr = np.frombuffer(rows[: min(cnt, cap) * ROW.itemsize].cpu().numpy().tobytes(), dtype=ROW).copy()
        log(f"traced 2^{lg} x {r} B k={k} {dist}: {len(tr)} rows, {int(((tr['flags'] & 1) != 0).sum())} sampled")
        out.append(tr)
        if per_workload is not None:
            per_workload.append(((lg, r, k, dist), tr))
        del data, tmp
        # give the cached blocks back: the library allocates its workspace
        # outside torch, and the 2^32-record workloads need most of the GPU
        torch.cuda.empty_cache()
    return np.concatenate(out) if out else np.zeros(0, dtype=ROW)


def dataset(tr):
    """Features, log2-time targets and masks of the sampled trace rows.

    Only sampled rows are used: each of them timed every feasible procedure
    under the same conditions (its input copied to tmp, one untimed run
    first).  The other rows time only the procedure the running scheduler
    chose, under other conditions (records already staged, the next job's
    loads in flight), so their targets would be confounded with that choice."""
    tr = tr[(tr["flags"] & 1) != 0]
    X = tr["features"].astype(np.float32)
    obs = tr["observed"].astype(np.uint32)
    M = np.stack([(obs >> q) & 1 for q in range(P)], axis=1).astype(np.float32)
    T = np.log2(tr["ticks"].astype(np.float64) + 1.0).astype(np.float32) * M
    return X, T, M


def balanced(parts, cap, seed=5):
    """The sampled rows of every workload, at most `cap` of each (a random
    subset), so that the largest sorts do not outweigh the others."""
    rng = np.random.default_rng(seed)
    out = []
    for _, tr in parts:
        s = tr[(tr["flags"] & 1) != 0]
        if len(s) > cap:
            s = s[np.sort(rng.choice(len(s), cap, replace=False))]
        out.append(s)
    return np.concatenate(out) if out else np.zeros(0, dtype=ROW)


def init_theta(rng, bias):
    def layer(o, i):
        return rng.normal(0.0, math.sqrt(2.0 / i), (o, i)), np.zeros(o)
    W1, b1 = layer(H, F)
    W2, b2 = layer(H, H)
    W3, _ = layer(P, H)
    W3 *= 0.1
    b3 = np.asarray(bias, dtype=np.float64)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3]).astype(np.float32)


def train(X, T, M, steps=3000, batch=4096, lr=2e-3, seed=7):
    """Adam on the masked MSE, in the library's kernels.  Returns (theta,
    mean, scale, loss history)."""
    import torch
    mean = X.mean(axis=0)
    scale = X.std(axis=0)
    scale = np.where(scale > 1e-3, scale, 1.0).astype(np.float32)
    Xn = ((X - mean) / scale).astype(np.float32)
    bias = [(T[:, q] * M[:, q]).sum() / max(M[:, q].sum(), 1.0) for q in range(P)]
    rng = np.random.default_rng(seed)
    dX = torch.from_numpy(Xn).cuda()
    dT = torch.from_numpy(T).cuda()
    dM = torch.from_numpy(M).cuda()
    theta = torch.from_numpy(init_theta(rng, bias)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = dX.shape[0]
    hist = []
    for t in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), device="cuda", generator=gen)
        xb, tb, mb = dX[idx].contiguous(), dT[idx].contiguous(), dM[idx].contiguous()
        raduls.mlp_loss_grad(xb, tb, mb, theta, grad, loss)
        raduls.mlp_adam(theta, grad, m, v, t, lr)
        if t % 250 == 0 or t == 1:
            hist.append((t, float(loss.cpu()[0])))
    return theta.cpu().numpy(), mean, scale, hist


def predict(theta, mean, scale, X):
    import torch
    Xn = torch.from_numpy(((X - mean) / scale).astype(np.float32)).cuda()
    Y = torch.empty((X.shape[0], P), dtype=torch.float32, device="cuda")
    raduls.mlp_forward(Xn, torch.from_numpy(np.asarray(theta, dtype=np.float32)).cuda(), Y)
    return Y.cpu().numpy()


def masked_argmin(Y, feas):
    big = np.float32(np.inf)
    Z = np.where(np.stack([(feas >> q) & 1 for q in range(P)], axis=1) > 0, Y, big)
    return Z.argmin(axis=1)


def regret(chosen, times, feas):
    """sum(t(chosen) - min t) / sum(min t) over rows with every feasible time."""
    t = times.astype(np.float64)
    ok = np.stack([(feas >> q) & 1 for q in range(P)], axis=1) > 0
    best = np.where(ok, t, np.inf).min(axis=1)
    got = t[np.arange(len(t)), chosen]
    return float((got - best).sum() / best.sum())


def evaluate(theta, mean, scale, tr):
    """Regret of the learned and of the recorded (running) choices on sampled rows."""
    s = tr[(tr["flags"] & 1) != 0]
    if len(s) == 0:
        return {"rows": 0}
    feas = s["observed"].astype(np.uint32)
    X = s["features"].astype(np.float32)
    Y = predict(theta, mean, scale, X)
    learned = masked_argmin(Y, feas)
    # outside the training range the sorter keeps the heuristic's choice
    ood = np.abs((X - mean) / scale).max(axis=1) > OOD_Z
    learned = np.where(ood, s["chosen"].astype(np.int64), learned)
    return {"rows": int(len(s)),
            "regret_learned": regret(learned, s["ticks"], feas),
            "regret_heuristic": regret(s["chosen"].astype(np.int64), s["ticks"], feas),
            "learned_picks": np.bincount(learned, minlength=P).tolist(),
            "out_of_range_rows": int(ood.sum()),
            "heuristic_picks": np.bincount(s["chosen"].astype(np.int64), minlength=P).tolist()}


def save_fixture(tr, path, rows=6000, seed=11):
    """A random subset of the sampled held-out rows (features, feasible set,
    per-procedure ticks, the heuristic's choice, job size), for an offline
    check of the trained network's regret."""
    s = tr[(tr["flags"] & 1) != 0]
    if len(s) > rows:
        s = s[np.sort(np.random.default_rng(seed).choice(len(s), rows, replace=False))]
    np.savez_compressed(path, features=s["features"].astype(np.float32), observed=s["observed"].astype(np.uint32),
                        ticks=s["ticks"].astype(np.uint32), chosen=s["chosen"].astype(np.uint32),
                        count=s["count"].astype(np.uint32), flags=s["flags"].astype(np.uint32))


def compare(blob, configs, reps=5, seed=500):
    """Median whole-sort ms, heuristic vs learned, per (log2 n, r, k, dist)."""
    import torch
    out = []
    for i, (lg, r, k, dist) in enumerate(configs):
        pristine = _inputs(lg, r, k, dist, seed + i)
        rec = torch.empty_like(pristine)
        tmp = torch.empty_like(pristine)
        res = {"config": f"2^{lg} x {r} B, k={k}, {dist}"}
        for label in ("heuristic", "learned"):
            if label == "learned":
                raduls.load_model(blob)
                raduls.set_scheduler(raduls.SCHED_LEARNED)
            else:
                raduls.set_scheduler(raduls.SCHED_HEURISTIC)
            raduls.set_timing(1)
            ts = []
            for _ in range(reps + 1):
                rec.copy_(pristine)
                torch.cuda.synchronize()
                raduls.sort(rec, k, tmp)
                torch.cuda.synchronize()
                ts.append(raduls.get_stats().last_ms)
            res[label + "_ms"] = float(np.median(ts[1:]))
        raduls.set_scheduler(raduls.SCHED_HEURISTIC)
        raduls.unload_model()
        res["learned_over_heuristic"] = res["heuristic_ms"] / res["learned_ms"]
        log(f"{res['config']}: heuristic {res['heuristic_ms']:.2f} ms, learned {res['learned_ms']:.2f} ms")
        out.append(res)
        del pristine, rec, tmp
    return out


def regret_report(workload, blob, seed=700, period=3):
    """Regret of the heuristic (the choices the traced sort made) and of the
    network `blob` (evaluated on the same sampled rows) for one workload."""
    theta, mean, scale = parse_blob(blob)
    lg, r, k, dist = workload
    tr = collect([workload], period, seed=seed, cap=1 << 23)
    e = evaluate(theta, mean, scale, tr)
    e.update({"workload": list(workload), "rows": int(len(tr))})
    return e


def parse_blob(blob: bytes):
    """(theta, mean, scale) of a model blob written by raduls.model_blob."""
    import struct
    f, h, p_ = struct.unpack("<3I", blob[8:20])
    a = np.frombuffer(blob[20:-4], dtype="<f4")
    n = f * h + h + h * h + h + p_ * h + p_
    return a[:n].copy(), a[n:n + f].copy(), a[n + f:n + 2 * f].copy()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--regret-workload", default="",
                    help="log2n,rec_bytes,key_bytes,dist: only report the regret of the committed network there")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--period", type=int, default=3)
    ap.add_argument("--compare-log2n", type=int, default=29)
    ap.add_argument("--per-workload", type=int, default=100_000, help="sampled training rows kept per workload")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    if args.regret_workload:
        lg, r, k, dist = args.regret_workload.split(",")
        with open(MODEL_PATH, "rb") as f:
            blob = f.read()
        raduls.set_scheduler(raduls.SCHED_HEURISTIC)
        rep = regret_report((int(lg), int(r), int(k), dist), blob)
        with open(os.path.join(args.out, "regret_report.json"), "w") as f:
            json.dump(rep, f, indent=1)
        print(json.dumps(rep), flush=True)
        return
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    raduls.unload_model()
    t0 = time.time()
    tr_parts = []
    tr = collect(TRAIN, args.period, seed=100, per_workload=tr_parts)
    ho_parts = []
    ho = collect(HOLDOUT, args.period, seed=300, per_workload=ho_parts)
    X, T, M = dataset(balanced(tr_parts, args.per_workload))
    log(f"{len(tr)} training rows, {len(ho)} held-out rows; training")
    theta, mean, scale, hist = train(X, T, M, steps=args.steps)
    blob = raduls.model_blob(theta, mean, scale)
    with open(os.path.join(args.out, "sched_mlp.rdls"), "wb") as f:
        f.write(blob)
    save_fixture(ho, os.path.join(args.out, "sched_holdout.npz"))
    ev_train = evaluate(theta, mean, scale, tr)
    ev_hold = evaluate(theta, mean, scale, ho)
    per = []
    for (w, part) in ho_parts:
        e = evaluate(theta, mean, scale, part)
        s_ = part[(part["flags"] & 1) != 0]
        mean_ticks = []
        for q in range(P):
            sel = ((s_["observed"] >> q) & 1) != 0
            mean_ticks.append(float(s_["ticks"][sel, q].mean()) if sel.any() else None)
        e.update({"workload": list(w), "mean_ticks_per_proc": mean_ticks,
                  "median_job_records": float(np.median(s_["count"])) if len(s_) else None})
        per.append(e)
    log(f"held-out regret: learned {ev_hold['regret_learned']:.4f}, heuristic {ev_hold['regret_heuristic']:.4f}")
    lg = args.compare_log2n
    cmp_ = compare(blob, [(lg, 16, 8, d) for d in ("uniform", "zipf", "prefix", "mix")] +
                   [(lg - 1, 32, 16, "zipf"), (lg, 8, 8, "mix")])
    report = {"train_rows": int(len(tr)), "fit_rows": int(len(X)), "holdout_rows": int(len(ho)), "loss_history": hist,
              "train_eval": ev_train, "holdout_eval": ev_hold, "holdout_per_workload": per, "end_to_end": cmp_,
              "train_workloads": [list(w) for w in TRAIN], "holdout_workloads": [list(w) for w in HOLDOUT],
              "seconds": time.time() - t0}
    with open(os.path.join(args.out, "learn_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps({"holdout_eval": ev_hold, "end_to_end": cmp_}), flush=True)


if __name__ == "__main__":
    main()
