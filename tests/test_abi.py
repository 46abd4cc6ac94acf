"""The C-ABI library without a GPU: it loads, exports every function the
header declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raduls.h")


@pytest.fixture(scope="module")
def R():
    from paper_1612_02557_amd import raduls
    if not os.path.exists(raduls.LIB_PATH):
        pytest.fail(f"{raduls.LIB_PATH} is not built (run __graft_entry__.build())")
    raduls.lib()
    return raduls


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"\b(raduls_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("raduls_sort", "raduls_sort_segmented", "raduls_partition", "raduls_set_scheduler",
                 "raduls_load_model", "raduls_get_stats", "raduls_workspace_bytes", "raduls_status_string",
                 "raduls_release", "raduls_mlp_forward", "raduls_mlp_loss_grad", "raduls_mlp_adam"):
        assert must in names


def test_library_exports_every_declared_function(R):
    L = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"declared but not exported: {missing}"
    assert set(declared_functions()) <= set(R.EXPORTS), "binding lacks a declared function"


def test_shape_validation(R):
    p = 1 << 20  # any 16-byte aligned non-null value: rejected before use
    assert R.sort_ptr(p, p + (1 << 30), 100, 6, 4, 0) == R.EUNSUPPORTED     # rec_bytes % 4
    assert R.sort_ptr(p, p + (1 << 30), 100, 16, 0, 0) == R.EINVAL          # key_bytes == 0
    assert R.sort_ptr(p, p + (1 << 30), 100, 8, 12, 0) == R.EINVAL          # key_bytes > rec_bytes
    assert R.sort_ptr(p, p + (1 << 30), 100, 32, 17, 0) == R.EUNSUPPORTED   # key_bytes > 16
    assert R.sort_ptr(p, p + (1 << 30), 100, 68, 8, 0) == R.EUNSUPPORTED    # rec_bytes > 64
    assert R.sort_ptr(0, 0, 100, 16, 8, 0) == R.EINVAL                      # null buffers
    assert R.sort_ptr(p, p + 800, 100, 16, 8, 0) == R.EINVAL                # records and tmp overlap
    assert R.sort_ptr(p + 4, p + (1 << 30), 100, 16, 8, 0) == R.EINVAL      # misaligned
    assert R.sort_ptr(p, p + (1 << 30), 1 << 40, 16, 8, 0) == R.EUNSUPPORTED
    assert R.sort_ptr(0, 0, 1, 16, 8, 0) == R.OK                            # n <= 1: nothing to do
    assert R.sort_ptr(0, 0, 0, 16, 8, 0) == R.OK


def test_segmented_and_partition_validation(R):
    L = R.lib()
    p = 1 << 20
    assert L.raduls_sort_segmented(p, p + (1 << 30), None, 3, 100, 16, 8, None) == R.EINVAL
    assert L.raduls_sort_segmented(p, p + (1 << 30), p + (1 << 31) + 4, 3, 100, 16, 8, None) == R.EINVAL
    assert L.raduls_sort_segmented(0, 0, 0, 0, 0, 16, 8, None) == R.OK
    assert L.raduls_partition(p, p + (1 << 30), 100, 16, 8, 0, 12, None, None) == R.EINVAL   # bits > 11
    assert L.raduls_partition(p, p + (1 << 30), 100, 16, 8, 64, 8, None, None) == R.EINVAL   # shift >= 64


def test_tuning_validation_and_roundtrip(R):
    t = R.default_tuning(16, 8, 1 << 30)
    assert t.big_digit_bits == 8 and t.tile_records == 4096
    R.set_tuning(t)
    got = R.get_tuning()
    assert got.as_dict() == t.as_dict()
    for field, bad in (("big_digit_bits", 12), ("block_digit_bits", 0), ("tile_records", 3000),
                       ("workgroups_per_cu", 9), ("big_rule", 2), ("job_records", 10)):
        b = R.default_tuning(16, 8, 1 << 20)
        setattr(b, field, bad)
        with pytest.raises(R.RadulsError) as e:
            R.set_tuning(b)
        assert e.value.code == R.EINVAL, field
    R.set_tuning(None)
    assert R.get_tuning() is None


def test_model_blob_validation_on_host(R):
    F, H, P = R.MLP_F, R.MLP_H, R.MLP_P
    theta = np.zeros(R.MLP_PARAMS, dtype=np.float32)
    good = R.model_blob(theta, np.zeros(F), np.ones(F))
    assert R.load_model_raw(good) == R.OK
    assert R.load_model_raw(good[:-1]) == R.EMODEL
    assert R.load_model_raw(b"RDLSMLP2" + good[8:]) == R.EMODEL
    bad = bytearray(good)
    bad[100] ^= 0x40
    assert R.load_model_raw(bytes(bad)) == R.EMODEL
    assert R.load_model_raw(R.model_blob(theta, np.zeros(F), -np.ones(F))) == R.EMODEL
    R.unload_model()


def test_scheduler_modes(R):
    R.set_scheduler(R.SCHED_FORCED, R.PROC_BITONIC)
    assert R.get_scheduler() == (R.SCHED_FORCED, R.PROC_BITONIC)
    R.set_scheduler(R.SCHED_HEURISTIC)
    assert R.get_scheduler()[0] == R.SCHED_HEURISTIC
    assert R.lib().raduls_set_scheduler(7, 0) == R.EINVAL


def test_status_strings_and_workspace(R):
    for code in (R.OK, R.EINVAL, R.ENOMEM, R.EHIP, R.EUNSUPPORTED, R.EMODEL, R.EDEVICE):
        s = R.status_string(code)
        assert s and s != "unknown status"
    assert R.status_string(12345) == "unknown status"
    a = R.workspace_bytes(1 << 20, 16, 8)
    b = R.workspace_bytes(1 << 26, 16, 8)
    assert 0 < a < b
    assert R.workspace_bytes(1 << 20, 6, 4) == 0


def test_mlp_entry_validation(R):
    L = R.lib()
    assert L.raduls_mlp_forward(None, None, None, 4, None) == R.EINVAL
    assert L.raduls_mlp_forward(None, None, None, 0, None) == R.OK
    assert L.raduls_mlp_adam(1 << 20, 1 << 21, 1 << 22, 1 << 23, 0, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                             ctypes.c_float(0.999), ctypes.c_float(1e-8), None) == R.EINVAL   # t counts from 1


def test_tune_validation(R):
    assert R.lib().raduls_tune(6, 4, 1 << 20, None) == R.EUNSUPPORTED
    assert R.lib().raduls_tune(16, 0, 1 << 20, None) == R.EINVAL


def test_digit_width_too_small_for_key_refused(R):
    """A tuning whose digit width would need more multi-workgroup levels than
    the plan holds (20) is refused before any device work: 16-byte keys at 6
    bits need 23, 8-byte keys at 3 bits need 23."""
    p = 1 << 20
    t = R.default_tuning(32, 16, 1 << 20)
    try:
        t.big_digit_bits = 6
        R.set_tuning(t)
        assert R.sort_ptr(p, p + (1 << 30), 100, 32, 16, 0) == R.EUNSUPPORTED
        assert "big_digit_bits" in R.lib().raduls_last_error_message().decode()
        t.big_digit_bits = 3
        R.set_tuning(t)
        assert R.sort_ptr(p, p + (1 << 30), 100, 16, 8, 0) == R.EUNSUPPORTED
        assert R.lib().raduls_sort_segmented(p, p + (1 << 30), p + (1 << 31), 3, 100, 16, 8, None) == R.EUNSUPPORTED
    finally:
        R.set_tuning(None)


def test_noalloc_validation(R):
    f = R.lib().raduls_sort_noalloc
    p = 1 << 20
    assert f(p, p + (1 << 30), 100, 6, 4, 0) == R.EUNSUPPORTED     # rec_bytes % 4
    assert f(p, p + (1 << 30), 100, 16, 0, 0) == R.EINVAL          # key_bytes == 0
    assert f(0, 0, 100, 16, 8, 0) == R.EINVAL                      # null buffers
    assert f(p, p + 800, 100, 16, 8, 0) == R.EINVAL                # records and tmp overlap
    assert f(p + 4, p + (1 << 30), 100, 16, 8, 0) == R.EINVAL      # misaligned
    assert f(0, 0, 1, 16, 8, 0) == R.OK                            # n <= 1: nothing to do


def test_count_runs_validation(R):
    p = 1 << 20
    G = 1 << 30
    ok_args = (p, 100, 16, 8, p + G, p + 2 * G, p + 3 * G, 0)
    call = R.count_runs_ptr
    assert call(p, 100, 6, 4, p + G, p + 2 * G, p + 3 * G, 0) == R.EUNSUPPORTED       # rec_bytes % 4
    assert call(p, 100, 16, 0, p + G, p + 2 * G, p + 3 * G, 0) == R.EINVAL            # key_bytes == 0
    assert call(p, 100, 16, 8, p + G, p + 2 * G, 0, 0) == R.EINVAL                    # null num_runs
    assert call(0, 100, 16, 8, p + G, p + 2 * G, p + 3 * G, 0) == R.EINVAL            # null records
    assert call(p, 100, 16, 8, p + G, 0, p + 3 * G, 0) == R.EINVAL                    # null counts
    assert call(p, 100, 16, 8, p + 16, p + 2 * G, p + 3 * G, 0) == R.EINVAL           # uniq overlaps partly
    assert call(p, 100, 16, 8, p + G, p + 800, p + 3 * G, 0) == R.EINVAL              # counts inside records
    assert call(p, 100, 16, 8, p + G, p + 2 * G, p + 2 * G + 8, 0) == R.EINVAL        # num_runs inside counts
    assert call(p + 4, 100, 16, 8, p + G, p + 2 * G, p + 3 * G, 0) == R.EINVAL        # misaligned records
    assert call(p, 100, 16, 8, p + G, p + 2 * G + 4, p + 3 * G, 0) == R.EINVAL        # misaligned counts
    assert call(p, 1 << 40, 16, 8, p + G, p + 2 * G, p + 3 * G, 0) == R.EUNSUPPORTED
    assert ok_args[0] == p



def test_prefix_search_validation(R):
    p = 1 << 20
    G = 1 << 30
    call = R.prefix_search_ptr
    # text, text_len, sa, queries, nq, rec_bytes, key_bytes, lo, hi, flags, stream
    assert call(p, 100, p + G, p + 2 * G, 10, 6, 4, p + 3 * G, p + 4 * G, 0, 0) == R.EUNSUPPORTED   # rec_bytes % 4
    assert call(p, 100, p + G, p + 2 * G, 10, 16, 0, p + 3 * G, p + 4 * G, 0, 0) == R.EINVAL        # key_bytes 0
    assert call(p, 100, p + G, p + 2 * G, 10, 16, 8, p + 3 * G, p + 4 * G, 2, 0) == R.EINVAL        # flags
    assert call(0, 100, p + G, p + 2 * G, 10, 16, 8, p + 3 * G, p + 4 * G, 0, 0) == R.EINVAL        # null text
    assert call(p, 0, p + G, p + 2 * G, 10, 16, 8, p + 3 * G, p + 4 * G, 0, 0) == R.EUNSUPPORTED    # empty text
    assert call(p, 1 << 32, p + G, p + 2 * G, 10, 16, 8, p + 3 * G, p + 4 * G, 0, 0) == R.EUNSUPPORTED
    assert call(p, 100, p + G, p + 2 * G + 4, 10, 16, 8, p + 3 * G, p + 4 * G, 0, 0) == R.EINVAL    # misaligned queries
    assert call(p, 100, p + G, p + 2 * G, 10, 16, 8, p + 3 * G, p + 3 * G + 40, 0, 0) == R.EINVAL   # lo and hi overlap
    assert call(p, 100, p + G, p + 2 * G, 10, 16, 8, p + 2 * G + 64, p + 4 * G, 0, 0) == R.EINVAL   # lo inside queries
    assert call(0, 0, 0, 0, 0, 16, 8, 0, 0, 0, 0) == R.OK                                           # no queries


def test_inplace_validation_and_workspace(R):
    f = R.sort_inplace_ptr
    p = 1 << 20
    assert f(p, 100, 6, 4, 0) == R.EUNSUPPORTED     # rec_bytes % 4
    assert f(p, 100, 16, 0, 0) == R.EINVAL          # key_bytes == 0
    assert f(p, 100, 8, 12, 0) == R.EINVAL          # key_bytes > rec_bytes
    assert f(p, 100, 68, 8, 0) == R.EUNSUPPORTED    # rec_bytes > 64
    assert f(0, 100, 16, 8, 0) == R.EINVAL          # null records
    assert f(p + 4, 100, 16, 8, 0) == R.EINVAL      # misaligned
    assert f(p, 1 << 40, 16, 8, 0) == R.EUNSUPPORTED
    assert f(0, 1, 16, 8, 0) == R.OK                # n <= 1: nothing to do
    assert f(0, 0, 16, 8, 0) == R.OK
    # the workspace replaces tmp at a fraction of its size
    n = 1 << 30
    w = R.inplace_workspace_bytes(n, 16, 8)
    assert 0 < w < n * 16 // 4
    assert w < R.workspace_bytes(n, 16, 8)
    assert R.inplace_workspace_bytes(n, 6, 4) == 0
