"""GPU tests of the other entry points against the oracle: the batched
segmented sort, one stable partition pass, the scheduler-network kernels,
the learned scheduler and the per-bucket trace."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp_ref, sched_ref
from synth import gen as sgen
from tests.gpu_util import first_diff, note, to_dev

pytestmark = pytest.mark.gpu

F, H, P = 9, 32, 3


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_1612_02557_amd import raduls
    assert torch.cuda.is_available()
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.set_tuning(None)
    raduls.unload_model()
    raduls.set_trace(None)
    yield raduls
    raduls.set_scheduler(raduls.SCHED_HEURISTIC)
    raduls.unload_model()
    raduls.set_trace(None)


# ---------------------------------------------------------------------------
# batched segmented sort

def seg_inputs(sizes, r, k, seed, payload="index"):
    sizes = np.asarray(sizes, dtype=np.uint64)
    off = synth.segment_offsets(sizes)
    dists = synth.segment_dists(len(sizes), seed)
    spec = synth.Spec(n=int(off[-1]), rec_bytes=r, key_bytes=k, payload=payload, seed=seed)
    return off, sgen.generate_segments(spec, off, dists)


def seg_check(R, host, off, k, label):
    import torch
    note(label)
    dev = to_dev(host)
    doff = torch.from_numpy(off.astype(np.int64)).to("cuda")
    R.sort_segmented(dev, doff, k)
    R.sync_check()
    got = dev.cpu().numpy()
    want = oracle.sort_segments(host, off, k)
    assert np.array_equal(got, want), f"{label}: {first_diff(got, want)}"


@pytest.mark.parametrize("S,lo,hi,seed", [(40, 1 << 4, 1 << 16, 1), (300, 1 << 2, 1 << 12, 2), (12, 1 << 10, 1 << 19, 3)])
def test_segmented_log_uniform(R, S, lo, hi, seed):
    sizes = synth.segment_sizes(S, seed, lo, hi)
    off, host = seg_inputs(sizes, 16, 8, seed)
    seg_check(R, host, off, 8, f"segmented S={S} sizes [{lo},{hi}) n={int(off[-1])}")


def test_segmented_edge_sizes(R):
    sizes = [0, 1, 2, 0, 33, 5000, 0, 1, 64, 65, 300_000, 3, 0]
    off, host = seg_inputs(sizes, 16, 8, 4)
    seg_check(R, host, off, 8, "segmented with empty and one-record segments")


def test_segmented_wide_records(R):
    sizes = synth.segment_sizes(25, 5, 1 << 6, 1 << 15)
    off, host = seg_inputs(sizes, 32, 16, 5, payload="random")
    seg_check(R, host, off, 16, "segmented r=32 k=16")


def test_segmented_one_segment_equals_sort(R):
    off, host = seg_inputs([1_000_003], 16, 8, 6)
    seg_check(R, host, off, 8, "segmented, a single segment of 1000003")


def test_segmented_replay_same_shape(R):
    """The second call with the same shape replays the captured graph on new data."""
    sizes = synth.segment_sizes(60, 7, 1 << 5, 1 << 14)
    for seed in (7, 8, 9):
        off = synth.segment_offsets(np.asarray(sizes, dtype=np.uint64))
        dists = synth.segment_dists(len(sizes), seed)
        host = sgen.generate_segments(synth.Spec(n=int(off[-1]), seed=seed), off, dists)
        seg_check(R, host, off, 8, f"segmented replay, data seed {seed}")


def test_segmented_bad_offsets_reported(R):
    import torch
    note("segmented with decreasing offsets")
    off, host = seg_inputs([100, 200, 300], 16, 8, 10)
    bad = off.copy().astype(np.int64)
    bad[1], bad[2] = 250, 120          # not non-decreasing
    dev = to_dev(host)
    R.sort_segmented(dev, torch.from_numpy(bad).to("cuda"), 8)
    with pytest.raises(R.RadulsError) as e:
        R.sync_check()
    assert e.value.code == R.EDEVICE
    assert np.array_equal(dev.cpu().numpy(), host), "data must be left unmodified"
    R.sync_check()                     # the flag is cleared


# ---------------------------------------------------------------------------
# one stable partition pass

@pytest.mark.parametrize("r,k,shift,bits,n", [(16, 8, 56, 8, 100_003), (16, 8, 0, 8, 70_001), (16, 8, 53, 11, 300_007),
                                           (16, 8, 30, 5, 4097), (16, 8, 63, 1, 65_537), (32, 16, 120, 8, 50_001),
                                           (8, 4, 24, 8, 1000), (12, 3, 5, 7, 9999)])
def test_partition(R, r, k, shift, bits, n):
    import torch
    note(f"partition r={r} k={k} shift={shift} bits={bits} n={n}")
    dist = "uniform" if k in (8, 16) else "bytes"
    host = synth.generate(synth.Spec(n=n, rec_bytes=r, key_bytes=k, dist=dist, payload="random", seed=n))
    src = to_dev(host)
    out = torch.empty_like(src)
    counts = torch.zeros(1 << bits, dtype=torch.int64, device="cuda")
    R.partition(src, out, k, shift, bits, counts)
    R.sync_check()
    want = oracle.partition(host, k, shift, bits)
    got = out.cpu().numpy()
    assert np.array_equal(got, want), first_diff(got, want)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint64), oracle.digit_histogram(host, k, shift, bits))
    assert np.array_equal(src.cpu().numpy(), host), "the input buffer is read only"


def test_wait_limit_reported(R, monkeypatch):
    """A look-back wait limit of 0 (a test-only setting read from the
    environment at planning time) makes every tile-offset chunk that
    continues a bucket give up at once.  Every kernel still exits, the
    scatters that would use the incomplete offsets are skipped, and the call
    reports EDEVICE through check=True; the next sort is exact again."""
    import torch
    note("look-back wait limit 0 -> EDEVICE")
    spec = synth.Spec(n=1 << 20, rec_bytes=16, key_bytes=8, dist="uniform", payload="index", seed=21)
    host = synth.generate(spec)
    dev = torch.from_numpy(host).to("cuda")
    monkeypatch.setenv("RADULS_TEST_SPIN_LIMIT", "0")
    with pytest.raises(R.RadulsError) as e:
        R.sort(dev, 8, check=True)
    assert e.value.code == R.EDEVICE
    assert "wait limit" in str(e.value)
    monkeypatch.delenv("RADULS_TEST_SPIN_LIMIT")
    dev = torch.from_numpy(host).to("cuda")
    R.sort(dev, 8, check=True)
    assert np.array_equal(dev.cpu().numpy(), oracle.sort(host, 8))


def test_check_option_passes_clean_sorts(R):
    import torch
    note("check=True on a clean sort and a clean segmented sort")
    off, host = seg_inputs([1000, 0, 5000], 16, 8, 12)
    dev = torch.from_numpy(host).to("cuda")
    R.sort_segmented(dev, torch.from_numpy(off.astype(np.int64)).to("cuda"), 8, check=True)
    assert np.array_equal(dev.cpu().numpy(), oracle.sort_segments(host, off, 8))


# ---------------------------------------------------------------------------
# scheduler-network kernels against the float64 reference

def mlp_case(seed, B):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.35, mlp_ref.n_params(F, H, P))
    X = rng.normal(0.0, 1.0, (B, F))
    T = rng.normal(0.0, 1.0, (B, P))
    M = (rng.random((B, P)) < 0.6).astype(np.float64)
    return theta, X, T, M


def f32dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


@pytest.mark.parametrize("B", [1, 37, 256, 4096])
def test_mlp_forward(R, B):
    import torch
    note(f"mlp forward B={B}")
    theta, X, _, _ = mlp_case(B, B)
    th32 = theta.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    Y = torch.empty((B, P), dtype=torch.float32, device="cuda")
    R.mlp_forward(f32dev(X32), f32dev(th32), Y)
    got = Y.cpu().numpy().astype(np.float64)
    want = mlp_ref.forward(th32, X32, F, H, P)
    # float32 evaluation of sums of at most 33 products of O(1) terms
    assert np.allclose(got, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())


def grad_error_bound(theta, X, T, M, gates, B):
    """Per-parameter bound on the float32 rounding error of the gradient.

    Each entry of the gradient is a sum over the batch, in index order, of
    products of forward and backward values.  A running-error analysis
    bounds its error by a multiple of u * S, u = 2^-24, where S is the same
    sum computed with every quantity replaced by the sum of the magnitudes
    it is formed from (Higham, Accuracy and Stability of Numerical
    Algorithms, Sec. 3.1 and 4.2).  The worst case multiple is the number
    of roundings K on the longest path: B - 1 additions of the batch sum
    plus at most 3 * (F + H + P) in the dot products behind one term.
    Rounding errors of independent-looking data add up like a random walk,
    so the multiple used is the probabilistic one, lambda * sqrt(K), with
    lambda = 8 (Higham and Mary, SIAM J. Sci. Comput. 41(5), 2019: it holds
    with probability at least 1 - 2 K exp(-lambda^2 / 2) per entry)."""
    u = 2.0 ** -24
    W1, b1, W2, b2, W3, b3 = (np.abs(a) for a in mlp_ref.unpack(theta, F, H, P))
    g1, g2 = gates
    xa = np.abs(X)
    h1a = np.where(g1, xa @ W1.T + b1, 0.0)
    h2a = np.where(g2, h1a @ W2.T + b2, 0.0)
    ya = h2a @ W3.T + b3
    s = max(float(M.sum()), 1.0)
    dya = 2.0 * M * (ya + np.abs(T)) / s
    da2a = np.where(g2, dya @ W3, 0.0)
    da1a = np.where(g1, da2a @ W2, 0.0)
    S = mlp_ref.pack(da1a.T @ xa, da1a.sum(axis=0), da2a.T @ h1a, da2a.sum(axis=0), dya.T @ h2a,
                     dya.sum(axis=0))
    K = (B - 1) + 3 * (F + H + P)
    return 8.0 * np.sqrt(K) * u * S


@pytest.mark.parametrize("B", [1, 64, 1000, 4096])
def test_mlp_loss_grad(R, B):
    import torch
    note(f"mlp loss/grad B={B}")
    theta, X, T, M = mlp_case(100 + B, B)
    th32, X32, T32 = (a.astype(np.float32).astype(np.float64) for a in (theta, X, T))
    grad = torch.empty(mlp_ref.n_params(F, H, P), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    R.mlp_loss_grad(f32dev(X32), f32dev(T32), f32dev(M), f32dev(th32), grad, loss)
    gates = mlp_ref.relu_gates_f32(th32, X32, F, H, P)
    L, g = mlp_ref.loss_and_grad(th32, X32, T32, M, F, H, P, relu_gate=gates)
    assert float(loss.cpu()[0]) == pytest.approx(L, rel=1e-4)
    gg = grad.cpu().numpy().astype(np.float64)
    # element by element, against the float32 error bound of each entry
    tol = grad_error_bound(th32, X32, T32, M, gates, B)
    bad = np.nonzero(np.abs(gg - g) > tol)[0]
    assert bad.size == 0, (f"{bad.size} gradient entries outside the bound, first {int(bad[0])}: "
                           f"{gg[bad[0]]!r} vs {g[bad[0]]!r} (bound {tol[bad[0]]:.3e})")


def test_mlp_empty_mask(R):
    import torch
    note("mlp loss/grad with an empty mask")
    theta, X, T, M = mlp_case(5, 128)
    grad = torch.full((mlp_ref.n_params(F, H, P),), 7.0, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    R.mlp_loss_grad(f32dev(X), f32dev(T), f32dev(np.zeros_like(M)), f32dev(theta), grad, loss)
    assert float(loss.cpu()[0]) == 0.0
    assert bool((grad == 0).all())


def test_mlp_adam(R):
    note("mlp adam, three steps")
    rng = np.random.default_rng(9)
    n = mlp_ref.n_params(F, H, P)
    th = rng.normal(0, 0.3, n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    dth, dm, dv = f32dev(th), f32dev(m), f32dev(v)
    # the kernel receives the hyper-parameters as float32; the reference
    # gets the same values
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-3, 0.9, 0.999, 1e-8))
    for t in (1, 2, 3):
        g = rng.normal(0, 1.0, n).astype(np.float32).astype(np.float64)
        R.mlp_adam(dth, f32dev(g), dm, dv, t, lr, b1, b2, eps)
        th, m, v = mlp_ref.adam_step(th, g, m, v, t, lr, b1, b2, eps)
        assert np.allclose(dth.cpu().numpy(), th, rtol=1e-5, atol=1e-6)
        assert np.allclose(dm.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
        assert np.allclose(dv.cpu().numpy(), v, rtol=1e-5, atol=1e-9)


# ---------------------------------------------------------------------------
# learned scheduler and trace

ROW = np.dtype([("features", "<f4", (9,)), ("chosen", "<u4"), ("count", "<u4"), ("observed", "<u4"),
                ("ticks", "<u4", (3,)), ("flags", "<u4")])


def traced_sort(R, host, k, cap=1 << 18, period=0):
    import torch
    rows = torch.zeros(cap * 64, dtype=torch.uint8, device="cuda")
    R.set_trace(rows, period)
    dev = to_dev(host)
    R.sort(dev, k)
    R.sync_check()
    cnt = R.trace_count()
    R.set_trace(None)
    got = dev.cpu().numpy()
    tr = np.frombuffer(rows.cpu().numpy().tobytes(), dtype=ROW)[:min(cnt, cap)].copy()
    return got, tr


def biased_model(prefer: int, seed: int = 0):
    """A network whose output for `prefer` is far below the others."""
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.05, mlp_ref.n_params(F, H, P))
    b3 = theta[-P:]
    b3[:] = 5.0
    b3[prefer] = -5.0
    # scales wide enough that every bucket is inside the training range
    return theta, np.zeros(F), np.full(F, 100.0)


OOD_Z = 4.0   # RADULS_MLP_OOD_Z


def heuristic_choice(row):
    """The paper's rule restricted to the feasible set of a counterfactual row."""
    m, feas = int(row["count"]), int(row["observed"])
    tiny = sched_ref.TINY_NARROW if row["features"][8] > 0.5 else sched_ref.TINY
    for q, ok in ((sched_ref.PROC_BITONIC, m < tiny), (sched_ref.PROC_RADIX, True), (sched_ref.PROC_LSD, True)):
        if ok and (feas >> q) & 1:
            return q
    return sched_ref.PROC_BITONIC


@pytest.mark.parametrize("dist", ["uniform", "zipf", "mix"])
def test_heuristic_trace_follows_rules(R, dist):
    note(f"heuristic trace, {dist}")
    host = synth.generate(synth.Spec(n=3_000_000, dist=dist, seed=21))
    got, tr = traced_sort(R, host, 8)
    assert np.array_equal(got, oracle.sort(host, 8))
    assert len(tr) > 0
    for row in tr[:20000]:
        m = int(row["count"])
        narrow = row["features"][8] > 0.5           # parent / m > 16, as the device decided it
        tiny = sched_ref.TINY_NARROW if narrow else sched_ref.TINY
        wave = bool(row["flags"] & 2)
        if m < tiny:
            want = sched_ref.PROC_BITONIC
        else:
            want = sched_ref.PROC_LSD if wave else sched_ref.PROC_RADIX
        assert int(row["chosen"]) == want, (m, bool(narrow), wave, int(row["chosen"]))
        lm = np.float32(np.log2(np.float32(m)))
        assert abs(row["features"][0] - lm) < 1e-5


@pytest.mark.parametrize("prefer", [sched_ref.PROC_LSD, sched_ref.PROC_BITONIC, sched_ref.PROC_RADIX])
def test_learned_scheduler_uses_network(R, prefer):
    note(f"learned scheduler preferring procedure {prefer}")
    theta, mean, scale = biased_model(prefer)
    R.load_model(R.model_blob(theta, mean, scale))
    R.set_scheduler(R.SCHED_LEARNED)
    try:
        host = synth.generate(synth.Spec(n=2_000_000, dist="mix", seed=22))
        got, tr = traced_sort(R, host, 8)
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)
        R.unload_model()
    assert np.array_equal(got, oracle.sort(host, 8)), "output must not depend on the scheduler"
    wave = (tr["flags"] & 2) != 0
    if prefer == sched_ref.PROC_RADIX:
        sel = ~wave               # RADIX is not feasible for wavefront jobs
    else:
        sel = np.ones(len(tr), dtype=bool)
    assert sel.sum() > 0
    assert np.all(tr["chosen"][sel] == prefer)


def test_learned_random_network_exact(R):
    note("learned scheduler with a random network")
    rng = np.random.default_rng(3)
    theta = rng.normal(0.0, 0.5, mlp_ref.n_params(F, H, P))
    R.load_model(R.model_blob(theta, rng.normal(0, 1, F), rng.uniform(0.5, 2.0, F)))
    R.set_scheduler(R.SCHED_LEARNED)
    try:
        for dist in ("uniform", "zipf", "prefix"):
            host = synth.generate(synth.Spec(n=1_500_000, dist=dist, seed=23))
            dev = to_dev(host)
            R.sort(dev, 8)
            R.sync_check()
            assert np.array_equal(dev.cpu().numpy(), oracle.sort(host, 8)), dist
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)
        R.unload_model()


def test_learned_choice_matches_host_network(R):
    """Counterfactual rows carry the feasible set; the device's choice is the
    masked argmin of the same network evaluated on the host in float32."""
    note("learned choice vs host float32 network")
    rng = np.random.default_rng(4)
    theta = rng.normal(0.0, 0.2, mlp_ref.n_params(F, H, P))
    theta[-P:] = [0.0, 1.5, -1.5]            # well separated outputs
    mean, scale = rng.normal(0, 0.5, F), rng.uniform(3.0, 6.0, F)
    R.load_model(R.model_blob(theta, mean, scale))
    R.set_scheduler(R.SCHED_LEARNED)
    try:
        host = synth.generate(synth.Spec(n=1_000_000, dist="mix", seed=24))
        got, tr = traced_sort(R, host, 8, period=1)
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)
        R.unload_model()
    assert np.array_equal(got, oracle.sort(host, 8))
    cf = tr[(tr["flags"] & 1) != 0]
    assert len(cf) > 0
    x = (cf["features"].astype(np.float32) - mean.astype(np.float32)) / scale.astype(np.float32)
    y = mlp_ref.forward_f32(theta, x, F, H, P)
    z = np.abs(x).max(axis=1)
    assert (z < OOD_Z - 1e-3).sum() > 0 and (z > OOD_Z + 1e-3).sum() > 0, "both sides of the range"
    for row, yy, zz in zip(cf, y, z):
        if abs(zz - OOD_Z) < 1e-3:
            continue                          # on the edge of the training range
        if zz > OOD_Z:
            assert int(row["chosen"]) == heuristic_choice(row), "outside the range: the heuristic decides"
            continue
        feas = int(row["observed"])
        cand = [q for q in range(P) if (feas >> q) & 1]
        best = min(cand, key=lambda q: (yy[q], q))
        srt = sorted(yy[q] for q in cand)
        if len(srt) > 1 and srt[1] - srt[0] < 1e-3:
            continue                          # too close to call across evaluation orders
        assert int(row["chosen"]) == best


def test_learned_out_of_range_falls_back(R):
    """A network whose training range (means and scales) excludes every
    bucket is never consulted: the choices are the heuristic's."""
    note("learned scheduler, buckets outside the training range")
    theta, _, _ = biased_model(sched_ref.PROC_LSD)
    mean = np.full(F, 1000.0)                 # z = (f - 1000) / 1 for features of order 1..30
    R.load_model(R.model_blob(theta, mean, np.ones(F)))
    R.set_scheduler(R.SCHED_LEARNED)
    try:
        host = synth.generate(synth.Spec(n=2_000_000, dist="mix", seed=26))
        got, tr = traced_sort(R, host, 8, period=1)
    finally:
        R.set_scheduler(R.SCHED_HEURISTIC)
        R.unload_model()
    assert np.array_equal(got, oracle.sort(host, 8))
    cf = tr[(tr["flags"] & 1) != 0]
    assert len(cf) > 0
    for row in cf[:5000]:
        assert int(row["chosen"]) == heuristic_choice(row)


def test_counterfactual_rows(R):
    note("counterfactual sampling, every job")
    host = synth.generate(synth.Spec(n=2_000_000, dist="zipf", seed=25))
    got, tr = traced_sort(R, host, 8, period=1)
    assert np.array_equal(got, oracle.sort(host, 8)), "timing every procedure must not change the output"
    cf = tr[(tr["flags"] & 1) != 0]
    assert len(cf) > 0
    for row in cf[:5000]:
        feas = int(row["observed"])
        assert bin(feas).count("1") >= 2
        assert (feas >> int(row["chosen"])) & 1
        for q in range(P):
            if (feas >> q) & 1:
                assert row["ticks"][q] > 0
    # regret of the heuristic's choices against the best observed procedure
    times = [[float(r["ticks"][q]) if (int(r["observed"]) >> q) & 1 else None for q in range(P)] for r in cf]
    reg = sched_ref.regret([int(r["chosen"]) for r in cf], times)
    assert reg >= 0.0


def test_model_blob_validation(R):
    note("model blob validation")
    theta, mean, scale = biased_model(1)
    good = R.model_blob(theta, mean, scale)
    assert R.load_model_raw(good) == R.OK
    bad_magic = b"X" + good[1:]
    assert R.load_model_raw(bad_magic) == R.EMODEL
    flipped = bytearray(good)
    flipped[40] ^= 1
    assert R.load_model_raw(bytes(flipped)) == R.EMODEL
    assert R.load_model_raw(good[:-1]) == R.EMODEL
    nan = R.model_blob(np.full_like(theta, np.nan), mean, scale)
    assert R.load_model_raw(nan) == R.EMODEL
    zero_scale = R.model_blob(theta, mean, np.zeros(F))
    assert R.load_model_raw(zero_scale) == R.EMODEL
    R.unload_model()


# ---------------------------------------------------------------------------
# autotuner

def test_autotuner_picks_a_valid_tuning(R):
    import time
    note("autotuner r=16 k=8 n_hint=2^22")
    R.set_tuning(None)
    t0 = time.perf_counter()
    t = R.tune(16, 8, 1 << 22)
    first = time.perf_counter() - t0
    try:
        assert t is not None
        d = t.as_dict()
        assert d["tile_records"] in (2048, 4096) and d["workgroups_per_cu"] in (1, 2)
        assert 8 <= d["big_digit_bits"] <= 11 and d["reg_finish"] in (0, 1)
        t0 = time.perf_counter()
        assert R.tune(16, 8, (1 << 22) + 5).as_dict() == d     # same size class: cached
        assert time.perf_counter() - t0 < first
        # the result applies to its shape and size class only
        assert R.effective_tuning(16, 8, (1 << 23) - 1).as_dict() == d
        assert R.effective_tuning(16, 8, 1 << 20).as_dict() == R.default_tuning(16, 8, 1 << 20).as_dict()
        assert R.effective_tuning(8, 8, 1 << 22).as_dict() == R.default_tuning(8, 8, 1 << 22).as_dict()
        for dist in ("uniform", "zipf"):
            host = synth.generate(synth.Spec(n=(1 << 22) + 12345, dist=dist, seed=31))
            dev = to_dev(host)
            R.sort(dev, 8)
            R.sync_check()
            assert np.array_equal(dev.cpu().numpy(), oracle.sort(host, 8)), dist
    finally:
        R.set_tuning(None)
    assert R.effective_tuning(16, 8, 1 << 22).as_dict() == R.default_tuning(16, 8, 1 << 22).as_dict()
