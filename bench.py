#!/usr/bin/env python3
"""Benchmark: sorted records/s of the MI355X MSD radix sort.

Workload (default): 2^30 records of 16 bytes -- 8-byte uniform random keys
from a seeded counter-based generator and an 8-byte payload holding each
record's original index -- sorted by raduls_sort on one GPU with the
heuristic scheduler.  The input is generated on the device, kept as a
pristine copy, and copied into the working buffer before every step
(outside the timed region), so every timed step sorts the same unsorted
input that is already resident in HBM.

Prints one JSON line: the metric, records/s, ms per step, the roofline of
the kernel with the most time per step (algorithmic bytes per launch over
its average launch time, against the 8 TB/s HBM peak), the end-to-end
fraction of the byte model, per-pass rates, the learned-scheduler leg and
the CPU oracle baseline.

Other legs: --batched (many independent arrays in one call vs one call per
array), --kmer (k-mer counting: sort + duplicate removal with counts, at the
sizes of the paper's three k-mer sets), --search (pattern-prefix search over
a suffix array, naive vs sorted queries), --inplace (the in-place variant,
no second buffer, against the out-of-place sort on the same input),
--autotune (the autotuner's tuning for the workload's shape against the
defaults).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published peak
METRIC = "sorted records/s and % of HBM roofline, 16-byte records, 1 MI355X; learned vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def model_bytes_per_record(n: int, r: int) -> float:
    """Algorithmic bytes per record of the method: r * (3 + 2P).

    One histogram read of the input, P multi-level partition passes of one
    read and one write each (the next level's histogram is counted with its
    pass), and one read plus one write by the LDS finishing sort; P is the
    number of 11-bit partition passes that bring buckets to the LDS
    finishing capacity of 64 KiB / r records.
    """
    import math
    cap = 65536 // r
    if n <= cap:
        return 2.0 * r
    P = math.ceil(math.log2(n / cap) / 11)
    return float(r * (3 + 2 * P))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_1612_02557_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(cs, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch from committed counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(f"{kernel}|{workload}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def host_description():
    """CPU model, logical CPUs and RAM of the host, from /proc."""
    model, ram = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_bytes": ram}


def cpu_baseline(pristine, key_bytes: int, sample_log2: int, single_log2: int):
    """The oracle (stable LSD byte-wise counting sort) on the host: threaded
    on the first 2^sample_log2 records, single-threaded on the first
    2^single_log2 records of the same input."""
    import numpy as np

    import oracle
    oracle.lib()
    cores = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        cores = max(1, min(cores, int(env)))

    def run(ns, threads):
        host = pristine[:ns].cpu().numpy().copy()
        t0 = time.perf_counter()
        oracle.sort_ref.sort_inplace(host, key_bytes, threads)
        dt = time.perf_counter() - t0
        k = host[:, :8].copy().view("<u8").ravel()
        assert bool(np.all(k[:-1] <= k[1:])), "oracle output not sorted"
        return dt

    ns = min(pristine.shape[0], 1 << sample_log2)
    dt = run(ns, cores)
    n1 = min(pristine.shape[0], 1 << single_log2)
    dt1 = run(n1, 1)
    return {"value": ns / dt, "unit": "records/s", "cores": cores, "kind": "oracle",
            "sample": f"first 2^{sample_log2} records of the benchmark input, stable LSD byte-wise counting sort "
                      f"in {cores} threads, {dt:.2f} s wall",
            "single_thread": {"value": n1 / dt1, "unit": "records/s", "cores": 1,
                              "sample": f"first 2^{single_log2} records, one thread, {dt1:.2f} s wall"},
            "host": host_description()}


def batched_check(rec, off, sizes, dists, spec, scratch, S):
    """Exactness of a segmented sort with payload = global index, chunk by chunk
    on the device: each output record equals the input record its payload
    names, that record lies in the same segment, and (key, payload) strictly
    increases inside each segment.  The input is regenerated into `scratch`."""
    import numpy as np
    import torch

    from synth import device as sdev
    s0 = 0
    while s0 < S:
        s1 = s0
        while s1 < S and int(off[s1 + 1]) - int(off[s0]) <= (1 << 27):
            s1 += 1
        s1 = max(s1, s0 + 1)
        a, b = int(off[s0]), int(off[s1])
        if b > a:
            sdev.generate_segments(spec, off, dists, out=scratch, segs=(s0, s1))
            o = rec[a:b].view(torch.int64).view(b - a, -1)
            key, idx = o[:, 0], o[:, 1]
            seg = torch.repeat_interleave(torch.arange(s1 - s0, device="cuda"),
                                          torch.from_numpy(sizes[s0:s1].astype(np.int64)).cuda())
            lo = torch.from_numpy(off[s0:s1].astype(np.int64)).cuda()[seg]
            hi = torch.from_numpy(off[s0 + 1:s1 + 1].astype(np.int64)).cuda()[seg]
            if not bool(((idx >= lo) & (idx < hi)).all()):
                return f"payload outside its segment in segments {s0}..{s1}"
            if not torch.equal(scratch[idx], rec[a:b]):
                return f"record differs from its input in segments {s0}..{s1}"
            ks = key ^ torch.iinfo(torch.int64).min
            same = seg[:-1] == seg[1:]
            ok = (ks[:-1] < ks[1:]) | ((ks[:-1] == ks[1:]) & (idx[:-1] < idx[1:]))
            if not bool((ok | ~same).all()):
                return f"order broken in segments {s0}..{s1}"
            del o, key, idx, seg, lo, hi, ks, same, ok
        s0 = s1
    return None


def batched_main(args):
    """Batched segmented sort (many independent arrays) in one call, against
    one raduls_sort call per array, on the same device-resident input."""
    import numpy as np
    import torch

    import synth
    from paper_1612_02557_amd import raduls
    from synth import device as sdev
    raduls.lib()
    S = args.segs
    sizes = synth.segment_sizes(S, args.seed, args.seg_lo, args.seg_hi)
    off = synth.segment_offsets(sizes)
    dists = synth.segment_dists(S, args.seed)
    n = int(off[-1])
    spec = synth.Spec(n=n, rec_bytes=16, key_bytes=8, payload="index", seed=args.seed)
    log(f"{S} segments, sizes log-uniform in [{args.seg_lo}, {args.seg_hi}], {n} records in all")
    rec = sdev.generate_segments(spec, off, dists)
    tmp = torch.empty_like(rec)
    doff = torch.from_numpy(off.astype(np.int64)).cuda()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        sdev.generate_segments(spec, off, dists, out=rec)
        torch.cuda.synchronize()
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def batched():
        raduls.sort_segmented(rec, doff, 8, tmp)

    def per_array():
        for s in range(S):
            a, b = int(off[s]), int(off[s + 1])
            if b - a > 1:
                raduls.sort(rec[a:b], 8, tmp[a:b])

    for _ in range(args.warmup):
        timed(batched)
    tb = [timed(batched) for _ in range(args.steps)]
    raduls.sync_check()
    err = batched_check(rec, off, sizes, dists, spec, tmp, S)
    if err:
        log(f"VERIFICATION FAILED: {err}")
    tuned_leg = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = raduls.tune(16, 8, n)
        tune_s = time.perf_counter() - t0
        timed(batched)
        tt = [timed(batched) for _ in range(args.steps)]
        raduls.sync_check()
        terr = batched_check(rec, off, sizes, dists, spec, tmp, S)
        mt = statistics.median(tt)
        tuned_leg = {"ms_per_step": mt, "value": n / (mt / 1e3), "default_over_tuned": statistics.median(tb) / mt,
                     "tuning": tuned.as_dict(), "tune_seconds": tune_s, "verified": terr is None, "step_ms": tt}
        log(f"batched, autotuned: {mt:.2f} ms")
        raduls.set_tuning(None)
    timed(per_array)
    tp = [timed(per_array) for _ in range(max(1, args.steps // 2))]
    mb, mp = statistics.median(tb), statistics.median(tp)
    out = {"metric": "batched segmented sort, records/s (one call vs one call per array)",
           "value": n / (mb / 1e3), "unit": "records/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": mb, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": f"{S} independent arrays of 16-byte records, sizes log-uniform in "
                                  f"[{args.seg_lo}, {args.seg_hi}], uniform or Zipf keys per array (seed {args.seed})",
                      "segments": S, "records": n},
           "per_array_ms": mp, "per_array_value": n / (mp / 1e3), "batched_over_per_array": mp / mb,
           "verified": err is None, "step_ms": tb, "per_array_step_ms": tp, "autotuned": tuned_leg}
    print(json.dumps(out), flush=True)


def kmer_main(args):
    """k-mer counting (paper, Sec. 5): records of 16 bytes whose 16-byte keys
    are 64-base k-mers of synthetic reads (one genome, coverage 16, one base
    in 64 records substituted), sorted and reduced to distinct k-mers with
    counts by raduls_sort_count, at the record counts of the paper's three
    k-mer sets.  Timed with HIP events on the stream the library uses; the
    run-counting kernel is also timed alone on the sorted records."""
    import numpy as np
    import torch

    import synth
    from paper_1612_02557_amd import raduls
    from synth import device as sdev
    raduls.lib()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_timing(0)
    sizes = [int(x) for x in args.kmer_sizes.split(",")]
    if args.autotune:
        t0 = time.perf_counter()
        for n in sizes:
            raduls.tune(16, 16, n)
        log(f"k-mers: autotuned in {time.perf_counter() - t0:.1f} s: "
            f"{[raduls.effective_tuning(16, 16, n).as_dict() for n in sizes]}")
    legs = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for n in sizes:
        spec = synth.Spec(n=n, rec_bytes=16, key_bytes=16, dist="kmer", payload="index", seed=args.seed)
        log(f"k-mers: generating {n} records")
        pristine = sdev.generate(spec)
        rec = torch.empty_like(pristine)
        tmp = torch.empty_like(pristine)
        counts = torch.empty(n, dtype=torch.int64, device="cuda")
        num = torch.empty(1, dtype=torch.int64, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        L = raduls.lib()

        def timed(fn):
            rec.copy_(pristine)
            torch.cuda.synchronize()
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1])

        def sort_count():
            raduls._check(L.raduls_sort_count(rec.data_ptr(), tmp.data_ptr(), n, 16, 16, tmp.data_ptr(),
                                              counts.data_ptr(), num.data_ptr(), st))

        for _ in range(args.warmup):
            timed(sort_count)
        t_all = [timed(sort_count) for _ in range(args.steps)]
        raduls.sync_check()
        U = int(num.item())
        # the run-counting kernel alone, on the sorted records now in `rec`
        raduls.sort(rec, 16, tmp)
        torch.cuda.synchronize()
        t_runs = []
        for _ in range(args.steps + 1):
            ev[0].record()
            raduls._check(L.raduls_count_runs(rec.data_ptr(), n, 16, 16, tmp.data_ptr(), counts.data_ptr(),
                                              num.data_ptr(), st))
            ev[1].record()
            torch.cuda.synchronize()
            t_runs.append(ev[0].elapsed_time(ev[1]))
        t_runs = t_runs[1:]
        raduls.sync_check()
        # checks that hold at any size: counts sum to n, positive, keys increase
        c = counts[:U]
        w = tmp[:U].view(torch.int64).view(U, 2)
        hi, lo = w[:, 1] ^ torch.iinfo(torch.int64).min, w[:, 0] ^ torch.iinfo(torch.int64).min
        inc = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))
        ok = int(c.sum().item()) == n and int(c.min().item()) >= 1 and bool(inc.all().item())
        ms, mr = statistics.median(t_all), statistics.median(t_runs)
        runs_bytes = 16 * n + U * (16 + 8)
        legs.append({"n": n, "distinct": U, "ms_sort_count": ms, "kmers_per_s": n / (ms / 1e3),
                     "ms_count_runs": mr, "count_runs_alg_bytes": runs_bytes,
                     "count_runs_GBps": runs_bytes / mr / 1e6, "count_runs_frac": runs_bytes / mr / 1e6 / HBM_PEAK_GBPS,
                     "sort_share": 1.0 - mr / ms, "verified": ok, "step_ms": t_all})
        log(f"k-mers n={n}: {ms:.2f} ms sort+count ({U} distinct), count alone {mr:.3f} ms")
        del pristine, rec, tmp, counts, num, c, w, hi, lo, inc
        torch.cuda.empty_cache()
    big = legs[-1]
    out = {"metric": "k-mers counted per second (sort + duplicate removal with counts), 16-byte k-mer records",
           "value": big["kmers_per_s"], "unit": "records/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": big["ms_sort_count"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
           "config": {"workload": "count the distinct 64-base k-mers (16-byte keys, 16-byte records) of synthetic "
                                  "reads of one genome, coverage 16, 1/64 records with a substituted base, at the "
                                  "record counts of the paper's three k-mer sets", "sizes": sizes,
                      "seed": args.seed},
           "roofline": {"bound": "hbm", "kernel": "k_runs", "achieved": big["count_runs_GBps"],
                        "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": big["count_runs_frac"], "traffic": None,
                        "alg_bytes_per_launch": big["count_runs_alg_bytes"], "avg_launch_ms": big["ms_count_runs"]},
           "legs": legs, "verified": all(l_["verified"] for l_ in legs),
           "tuning": ([raduls.effective_tuning(16, 16, n).as_dict() for n in sizes] if args.autotune else "default")}
    print(json.dumps(out), flush=True)


def search_main(args):
    """Batched pattern-prefix search (paper, Sec. 5): a text of 2^text_log2
    random DNA characters (two bits of the k-mer generator's genome stream per
    character), its suffix array (built here by raduls_sort of records keyed
    by each suffix's first 42 characters, 3 bits each, checked distinct), and
    2^q_log2 queries of 16 characters (three in four copied from random text
    positions, one in four random) as 24-byte records (reversed characters,
    then the query id).  Timed: one full binary search per query in input
    order (the naive way) against sorting the queries first and searching
    them in narrowed ranges (raduls_sort_search)."""
    import numpy as np
    import torch

    import synth
    from paper_1612_02557_amd import raduls
    from synth import device as sdev
    raduls.lib()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_timing(0)
    N, nq, K = 1 << args.text_log2, 1 << args.q_log2, 16
    log(f"search: text of {N} characters, {nq} queries of {K} characters")
    words = sdev.generate(synth.Spec(n=(N + 31) // 32, rec_bytes=8, key_bytes=8, dist="uniform", seed=args.seed))
    w = words.view(torch.int64).view(-1)
    text = torch.empty(((N + 31) // 32) * 32, dtype=torch.uint8, device="cuda")
    tv = text.view(-1, 32)
    for j in range(32):
        tv[:, j] = (((w >> (2 * j)) & 3) + 1).to(torch.uint8)
    text = text[:N].contiguous()
    del words, w, tv
    # suffix array: 126-bit keys of the first 42 characters (0 past the end)
    tp = torch.cat([text, torch.zeros(42, dtype=torch.uint8, device="cuda")]).to(torch.int64)
    lo = torch.zeros(N, dtype=torch.int64, device="cuda")
    hi = torch.zeros(N, dtype=torch.int64, device="cuda")
    for j in range(42):
        c = tp[j:j + N]
        b = 123 - 3 * j   # lowest bit of character j's field
        if b >= 64:
            hi |= c << (b - 64)
        elif b + 2 < 64:
            lo |= c << b
        else:   # the field straddles the words (b = 63): its low bit is lo's top bit
            lo |= torch.where((c & 1) == 1, torch.iinfo(torch.int64).min, 0)
            hi |= c >> (64 - b)
    rec = torch.empty((N, 24), dtype=torch.uint8, device="cuda")
    rv = rec.view(torch.int64).view(N, 3)
    rv[:, 0], rv[:, 1] = lo, hi
    rv[:, 2] = torch.arange(N, dtype=torch.int64, device="cuda")
    del tp, lo, hi
    raduls.sort(rec, 16, check=True)
    rv = rec.view(torch.int64).view(N, 3)
    ulo, uhi = rv[:, 0] ^ torch.iinfo(torch.int64).min, rv[:, 1] ^ torch.iinfo(torch.int64).min
    distinct = bool(((uhi[1:] > uhi[:-1]) | ((uhi[1:] == uhi[:-1]) & (ulo[1:] > ulo[:-1]))).all().item())
    sa = rv[:, 2].to(torch.int32).contiguous()
    del rec, rv, ulo, uhi
    torch.cuda.empty_cache()
    # queries
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    pos = torch.randint(0, N - K, (nq,), device="cuda", generator=g)
    qchars = text[pos.unsqueeze(1) + torch.arange(K, device="cuda")]
    rnd = torch.randint(1, 5, (nq, K), device="cuda", generator=g, dtype=torch.int64).to(torch.uint8)
    take = (torch.arange(nq, device="cuda") % 4 == 3).unsqueeze(1)
    qchars = torch.where(take, rnd, qchars)
    pristine = torch.zeros((nq, 24), dtype=torch.uint8, device="cuda")
    pristine[:, :K] = qchars.flip(1)
    pristine.view(torch.int64).view(nq, 3)[:, 2] = torch.arange(nq, dtype=torch.int64, device="cuda")
    del qchars, rnd, take, pos
    q = torch.empty_like(pristine)
    tmp = torch.empty_like(pristine)
    lo1 = torch.empty(nq, dtype=torch.int64, device="cuda")
    hi1 = torch.empty_like(lo1)
    lo2 = torch.empty_like(lo1)
    hi2 = torch.empty_like(lo1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        q.copy_(pristine)
        torch.cuda.synchronize()
        ev[0].record()
        fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])

    def naive():
        raduls.prefix_search(text, sa, q, K, lo=lo1, hi=hi1, narrow=False)

    def sorted_search():
        raduls.sort_search(text, sa, q, K, tmp=tmp, lo=lo2, hi=hi2)

    for _ in range(args.warmup):
        timed(naive)
        timed(sorted_search)
    tn = [timed(naive) for _ in range(args.steps)]
    ts = [timed(sorted_search) for _ in range(args.steps)]
    # the search alone on the sorted queries now in q
    t_alone = []
    for _ in range(args.steps):
        ev[0].record()
        raduls.prefix_search(text, sa, q, K, lo=lo2, hi=hi2)
        ev[1].record()
        torch.cuda.synchronize()
        t_alone.append(ev[0].elapsed_time(ev[1]))
    raduls.sync_check()
    # checks: both ways give the same range for every query (through the ids);
    # sampled ranges bound the matching suffixes (text gathers on the device)
    ids = q.view(torch.int64).view(nq, 3)[:, 2]
    same = bool(torch.equal(lo1[ids], lo2) and torch.equal(hi1[ids], hi2))
    smp = torch.randint(0, nq, (4096,), device="cuda", generator=g)
    qk = pristine[smp, :K].flip(1).to(torch.int64)             # characters in reading order

    def pref(rank):
        p = sa[rank.clamp(0, N - 1)].to(torch.int64)
        idx = p.unsqueeze(1) + torch.arange(K, device="cuda")
        c = text[idx.clamp(max=N - 1)].to(torch.int64)
        return torch.where(idx < N, c, torch.zeros_like(c))

    def cmp(a, b):   # -1, 0, 1 per row, first differing character decides
        d = torch.sign(a - b)
        first = torch.argmax((d != 0).to(torch.int8), dim=1)
        return d.gather(1, first.unsqueeze(1)).squeeze(1)

    l_, h_ = lo1[smp], hi1[smp]
    ok = bool((l_ <= h_).all().item())
    ok &= bool(((l_ == 0) | (cmp(pref(l_ - 1), qk) < 0)).all().item())
    ok &= bool(((l_ == N) | (cmp(pref(l_), qk) >= 0)).all().item())
    ok &= bool(((h_ == l_) | (cmp(pref(h_ - 1), qk) == 0)).all().item())
    ok &= bool(((h_ == N) | (cmp(pref(h_), qk) > 0)).all().item())
    found = int((hi1 > lo1).sum().item())
    mn, ms, ma = statistics.median(tn), statistics.median(ts), statistics.median(t_alone)
    io_bytes = nq * (24 + 16)
    out = {"metric": "patterns searched per second in a suffix array (sort + narrowed search), 16-character prefixes",
           "value": nq / (ms / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128",
           "data": "synthetic",
           "config": {"workload": f"{nq} queries of 16 characters (3/4 taken from the text, 1/4 random) against the "
                                  f"suffix array of 2^{args.text_log2} random DNA characters", "text": N,
                      "queries": nq, "seed": args.seed},
           "roofline": {"bound": "latency", "kernel": "k_prefix_search", "achieved": io_bytes / ma / 1e6,
                        "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": io_bytes / ma / 1e6 / HBM_PEAK_GBPS,
                        "traffic": None, "alg_bytes_per_launch": io_bytes, "avg_launch_ms": ma,
                        "note": "dependent random probes; the bytes are the queries read and the ranges written"},
           "naive_ms": mn, "naive_value": nq / (mn / 1e3), "sorted_over_naive": mn / ms, "search_alone_ms": ma,
           "queries_found": found, "suffixes_distinct": distinct, "verified": bool(same and ok and distinct),
           "step_ms": ts, "naive_step_ms": tn}
    log(f"search: naive {mn:.2f} ms, sort + search {ms:.2f} ms (search alone {ma:.2f} ms), {found} queries found")
    print(json.dumps(out), flush=True)


def inplace_main(args):
    """The in-place sort (raduls_sort_inplace) of the default workload, timed
    like the main leg, with per-phase rates, the roofline of the kernel with
    the most time per step, its memory next to the out-of-place sort's, and
    the out-of-place sort of the same input in the same run."""
    import torch

    import synth
    from paper_1612_02557_amd import raduls
    from synth import device as sdev
    from tests.gpu_util import unstable_index_check

    raduls.lib()
    n = 1 << args.log2n
    r, k = args.rec_bytes, args.key_bytes
    if r < k + 8 or k not in (8, 16):
        raise SystemExit("--inplace needs an 8- or 16-byte key followed by the 8-byte index payload")
    spec = synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=args.dist, payload="index", seed=args.seed)
    log(f"generating {n} x {r}-byte records ({args.dist}) on the device")
    pristine = sdev.generate(spec)
    rec = torch.empty_like(pristine)
    torch.cuda.synchronize()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    raduls.set_timing(2 if args.phases else 1)

    def step(fn):
        rec.copy_(pristine)
        torch.cuda.synchronize()
        fn()
        torch.cuda.synchronize()
        return raduls.get_stats().last_ms

    for w in range(args.warmup):
        log(f"warmup {w}: {step(lambda: raduls.sort_inplace(rec, k)):.3f} ms")
    times, phase_acc = [], {}
    for s_ in range(args.steps):
        ms = step(lambda: raduls.sort_inplace(rec, k))
        times.append(ms)
        if args.phases:
            for name, v in raduls.phase_times().items():
                phase_acc.setdefault(name, []).append(v)
        log(f"step {s_}: {ms:.3f} ms")
    work = raduls.last_work()
    ms_per_step = statistics.mean(times)
    err = unstable_index_check(rec, pristine, k)
    verified = err is None
    if err:
        log(f"VERIFICATION FAILED: {err}")
    try:
        raduls.sync_check()
    except raduls.RadulsError as e:
        log(f"device check failed: {e}")
        verified = False

    # algorithmic bytes: a level reads and writes its records twice (into
    # blocks, then the blocks into place): the records of the buckets split
    # into stripes by the classification and the permutation (2r each), the
    # others by the one-workgroup kernel (4r); finishing reads and writes once
    passes = []
    for l, (n_in, n_large) in enumerate(work["levels"]):
        n_med = n_in - n_large
        for kind, kern, recs, mult in (("hist", "k_ip_classify", n_large, 2), ("prep", "k_ip_medium", n_med, 4),
                                       ("scatter", "k_ip_permute", n_large, 2)):
            name = f"L{l}.{kind}"
            if name in phase_acc and recs:
                t = statistics.mean(phase_acc[name])
                b = mult * r * recs
                passes.append({"phase": name, "kernel": kern, "ms": t, "records": recs, "alg_bytes": b,
                               "GBps": b / t / 1e6 if t > 0 else None})
    if "small_jobs" in phase_acc:
        t = statistics.mean(phase_acc["small_jobs"])
        b = 2 * r * work["wg_jobs"]
        passes.append({"phase": "small_jobs", "kernel": "k_fin_jobs", "ms": t, "records": work["wg_jobs"],
                       "alg_bytes": b, "GBps": b / t / 1e6 if t > 0 else None})
    other = {nm: statistics.mean(v) for nm, v in phase_acc.items()
             if not any(p_["phase"] == nm for p_ in passes)}
    kernels = {}
    for p_ in passes:
        if not p_["ms"] or p_["records"] == 0:
            continue
        k_ = kernels.setdefault(p_["kernel"], {"launches": 0, "ms": 0.0, "alg_bytes": 0})
        k_["launches"] += 1
        k_["ms"] += p_["ms"]
        k_["alg_bytes"] += p_["alg_bytes"]
    for name, k_ in kernels.items():
        k_["avg_launch_ms"] = k_["ms"] / k_["launches"]
        k_["alg_bytes_per_launch"] = k_["alg_bytes"] / k_["launches"]
        k_["GBps"] = k_["alg_bytes"] / k_["ms"] / 1e6
    roof = None
    if kernels:
        dn, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
        wl = f"inplace-{args.dist}-2^{args.log2n}x{r}B"
        roof = {"bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": dom["GBps"] / HBM_PEAK_GBPS, "traffic": load_traffic(dn, wl),
                "kernel": dn, "launches_per_step": dom["launches"], "ms_per_step": dom["ms"],
                "avg_launch_ms": dom["avg_launch_ms"], "alg_bytes_per_launch": dom["alg_bytes_per_launch"]}

    # the out-of-place sort of the same input, for context
    tmp = torch.empty_like(pristine)
    oop = []
    for s_ in range(max(1, args.steps)):
        oop.append(step(lambda: raduls.sort(rec, k, tmp)))
    del tmp
    torch.cuda.empty_cache()
    ms_oop = statistics.mean(oop)
    mem = {"records_bytes": n * r, "inplace_workspace_bytes": raduls.inplace_workspace_bytes(n, r, k),
           "out_of_place_extra_bytes": n * r + raduls.workspace_bytes(n, r, k)}
    log(f"in place {ms_per_step:.2f} ms, out of place {ms_oop:.2f} ms; extra memory "
        f"{mem['inplace_workspace_bytes'] / 2**30:.2f} GiB vs {mem['out_of_place_extra_bytes'] / 2**30:.2f} GiB")
    out = {"metric": "records sorted per second in place (no second buffer), 16-byte records, 1 MI355X",
           "value": n / (ms_per_step / 1e3), "unit": "records/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64" if k == 8 else "u128", "data": "synthetic",
           "config": {"workload": f"in-place sort of 2^{args.log2n} {r}-byte records ({k}-byte {args.dist} keys, "
                                  f"8-byte index payload; not stable)", "seed": args.seed},
           "roofline": roof, "kernels": kernels, "passes": passes, "other_phases_ms": other,
           "memory": mem, "out_of_place_ms": ms_oop, "inplace_over_out_of_place_time": ms_per_step / ms_oop,
           "step_ms": times, "verified": verified}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=30)
    ap.add_argument("--rec-bytes", type=int, default=16)
    ap.add_argument("--key-bytes", type=int, default=8)
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample-log2", type=int, default=28)
    ap.add_argument("--cpu-single-log2", type=int, default=25)
    ap.add_argument("--phases", type=int, default=1, help="1: per-phase events during the timed steps")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-scheduler leg")
    ap.add_argument("--tuning", default="", help="tuning overrides, e.g. big_min=8192,workgroups_per_cu=3")
    ap.add_argument("--batched", action="store_true", help="batched segmented sort vs one call per array")
    ap.add_argument("--segs", type=int, default=10000)
    ap.add_argument("--seg-lo", type=int, default=1 << 10)
    ap.add_argument("--seg-hi", type=int, default=1 << 22)
    ap.add_argument("--kmer", action="store_true", help="k-mer counting: sort + duplicate removal with counts")
    ap.add_argument("--kmer-sizes", default="63000000,413000000,1887000000")
    ap.add_argument("--search", action="store_true", help="batched pattern-prefix search over a suffix array")
    ap.add_argument("--inplace", action="store_true", help="in-place sort (no second buffer) vs out of place")
    ap.add_argument("--text-log2", type=int, default=28)
    ap.add_argument("--q-log2", type=int, default=24)
    ap.add_argument("--autotune", action="store_true",
                    help="time the autotuner's tuning for this shape against the defaults")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the batched and single-array paths are single-GPU)", file=sys.stderr)
        sys.exit(2)

    if args.batched:
        return batched_main(args)
    if args.kmer:
        return kmer_main(args)
    if args.search:
        return search_main(args)
    if args.inplace:
        return inplace_main(args)

    import torch

    import synth
    from paper_1612_02557_amd import raduls
    from synth import device as sdev
    from tests.gpu_util import exact_index_check

    raduls.lib()
    n = 1 << args.log2n
    r, k = args.rec_bytes, args.key_bytes
    spec = synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=args.dist, payload="index", seed=args.seed)
    log(f"generating {n} x {r}-byte records ({args.dist}) on the device")
    pristine = sdev.generate(spec)
    rec = torch.empty_like(pristine)
    tmp = torch.empty_like(pristine)
    torch.cuda.synchronize()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_timing(2 if args.phases else 1)
    tuning = None
    if args.tuning:
        t = raduls.default_tuning(r, k, n)
        for kv in args.tuning.split(","):
            key, val = kv.split("=")
            if not hasattr(t, key):
                raise SystemExit(f"unknown tuning field {key}")
            setattr(t, key, int(val))
        raduls.set_tuning(t)
        tuning = t.as_dict()

    def step():
        rec.copy_(pristine)
        torch.cuda.synchronize()
        raduls.sort(rec, k, tmp)
        torch.cuda.synchronize()
        return raduls.get_stats().last_ms

    for w in range(args.warmup):
        ms = step()
        log(f"warmup {w}: {ms:.3f} ms")
    times, phase_acc = [], {}
    wall0 = time.perf_counter()
    for s in range(args.steps):
        ms = step()
        times.append(ms)
        if args.phases:
            for name, v in raduls.phase_times().items():
                phase_acc.setdefault(name, []).append(v)
        log(f"step {s}: {ms:.3f} ms")
    wall = time.perf_counter() - wall0
    work = raduls.last_work()
    ms_per_step = statistics.mean(times)
    value = n / (ms_per_step / 1e3)

    err = exact_index_check(rec, pristine, r, k)
    verified = None if err == "unchecked" else err is None
    if err and err != "unchecked":
        log(f"VERIFICATION FAILED: {err}")
    try:
        raduls.sync_check()
    except raduls.RadulsError as e:
        log(f"device check failed: {e}")
        verified = False

    # per-pass algorithmic bytes and rates
    passes = []
    for l, (n_in, n_moved) in enumerate(work["levels"]):
        for kind, kern, recs, mult in (("hist", "k_hist_wave", n_in, 1), ("scatter", "k_scatter", n_moved, 2)):
            name = f"L{l}.{kind}"
            if name in phase_acc:
                t = statistics.mean(phase_acc[name])
                b = mult * r * recs
                passes.append({"phase": name, "kernel": kern, "ms": t, "records": recs, "alg_bytes": b,
                               "GBps": b / t / 1e6 if t > 0 else None})
    # single-workgroup queue pass: a one-workgroup radix pass reads its bucket
    # twice (count, move) and writes it once; wavefront and tiny jobs read
    # and write once
    if "small" in phase_acc:
        t = statistics.mean(phase_acc["small"])
        recs = work["block_pass"] + work["wave_jobs"] + work["tiny_done"]
        b = r * (3 * work["block_pass"] + 2 * (work["wave_jobs"] + work["tiny_done"]))
        passes.append({"phase": "small", "kernel": "k_small", "ms": t, "records": recs, "alg_bytes": b,
                       "GBps": b / t / 1e6 if t > 0 else None})
    if "small_jobs" in phase_acc:
        t = statistics.mean(phase_acc["small_jobs"])
        recs = work["wg_jobs"]
        b = 2 * r * recs
        kern = "k_fin_jobs" if work.get("fin_max") else "k_small_jobs"
        passes.append({"phase": "small_jobs", "kernel": kern, "ms": t, "records": recs, "alg_bytes": b,
                       "GBps": b / t / 1e6 if t > 0 else None})
    other = {nm: statistics.mean(v) for nm, v in phase_acc.items()
             if not any(p["phase"] == nm for p in passes)}

    # per kernel: launches, time per step, algorithmic bytes; the dominant
    # kernel is the one with the most time per step (all its launches)
    kernels = {}
    for p_ in passes:
        if not p_["ms"] or p_["records"] == 0:
            continue
        k_ = kernels.setdefault(p_["kernel"], {"launches": 0, "ms": 0.0, "alg_bytes": 0})
        k_["launches"] += 1
        k_["ms"] += p_["ms"]
        k_["alg_bytes"] += p_["alg_bytes"]
    for name, k_ in kernels.items():
        k_["avg_launch_ms"] = k_["ms"] / k_["launches"]
        k_["alg_bytes_per_launch"] = k_["alg_bytes"] / k_["launches"]
        k_["GBps"] = k_["alg_bytes"] / k_["ms"] / 1e6
    roof = None
    if kernels:
        dn, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
        wl = f"{args.dist}-2^{args.log2n}x{r}B"
        tr = load_traffic(dn, wl)
        roof = {"bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": dom["GBps"] / HBM_PEAK_GBPS, "traffic": tr,
                "kernel": dn, "launches_per_step": dom["launches"], "ms_per_step": dom["ms"],
                "avg_launch_ms": dom["avg_launch_ms"], "alg_bytes_per_launch": dom["alg_bytes_per_launch"]}
    bpr = model_bytes_per_record(n, r)
    t_roof_ms = bpr * n / (HBM_PEAK_GBPS * 1e9) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if k == 8 else "u128",
        "data": "synthetic",
        "config": {"workload": f"sort 2^{args.log2n} records of {r} bytes, {args.dist} {k}-byte keys, "
                               f"payload = original index (seed {args.seed})",
                   "n": n, "rec_bytes": r, "key_bytes": k, "dist": args.dist, "seed": args.seed,
                   "scheduler": "heuristic", **({"tuning": tuning} if tuning else {})},
        "roofline": roof,
        "e2e": {"model_bytes_per_record": bpr, "t_roof_ms": t_roof_ms, "frac": t_roof_ms / ms_per_step,
                "model_GBps": bpr * n / (ms_per_step / 1e3) / 1e9},
        "passes": passes,
        "kernels": kernels,
        "other_phases_ms": other,
        "step_ms": times,
        "timed_wall_s": wall,
        "verified": verified,
    }
    # the autotuner's tuning for this shape, heuristic scheduler
    autotuned = None
    if args.autotune and not args.tuning:
        raduls.set_timing(1)
        t0 = time.perf_counter()
        tuned = raduls.tune(r, k, n)
        tune_s = time.perf_counter() - t0
        step()
        at = [step() for _ in range(args.steps)]
        aerr = exact_index_check(rec, pristine, r, k)
        ams = statistics.mean(at)
        autotuned = {"ms_per_step": ams, "value": n / (ams / 1e3), "default_over_tuned": ms_per_step / ams,
                     "tuning": tuned.as_dict(), "default": raduls.default_tuning(r, k, n).as_dict(),
                     "tune_seconds": tune_s, "verified": None if aerr == "unchecked" else aerr is None}
        log(f"autotuned: {ams:.3f} ms per step (tuning took {tune_s:.1f} s)")
    # learned scheduler on the same input (the committed trained network),
    # with the autotuned tuning when --autotune ran
    learned = None
    model = os.path.join(ROOT, "paper_1612_02557_amd", "models", "sched_mlp.rdls")
    if not args.no_learned and os.path.exists(model):
        with open(model, "rb") as f:
            raduls.load_model(f.read())
        raduls.set_scheduler(raduls.SCHED_LEARNED)
        raduls.set_timing(1)
        step()
        lt = [step() for _ in range(args.steps)]
        lerr = exact_index_check(rec, pristine, r, k)
        lok = None if lerr == "unchecked" else lerr is None
        raduls.set_scheduler(raduls.SCHED_HEURISTIC)
        raduls.unload_model()
        lms = statistics.mean(lt)
        learned = {"ms_per_step": lms, "value": n / (lms / 1e3), "unit": "records/s",
                   "plain_over_learned": ms_per_step / lms, "verified": lok,
                   "model": "paper_1612_02557_amd/models/sched_mlp.rdls"}
        log(f"learned scheduler: {lms:.3f} ms per step")
    out["learned"] = learned
    out["autotuned"] = autotuned
    del tmp, rec
    torch.cuda.empty_cache()
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(pristine, k, args.cpu_sample_log2, args.cpu_single_log2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
