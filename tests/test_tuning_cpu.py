"""Launch settings and the autotuner's results file, host side: the field
checks of sdd_validate_tuning and the file format of sdd_tune_cache_lookup /
sdd_tune_cache_store (no device needed)."""
import pytest

import paper_1912_06474_amd as m


@pytest.mark.parametrize("t", [dict(), dict(batch_paths=512), dict(batch_paths=1 << 24), dict(trace_grid=8),
                               dict(trace_grid=4096), dict(dir_bins=1), dict(dir_bins=4),
                               dict(batch_paths=1 << 20, trace_grid=512, dir_bins=1)])
def test_valid_tunings(t):
    ok, msg = m.validate_tuning(**t)
    assert ok and msg == ""


@pytest.mark.parametrize("t,word", [(dict(batch_paths=511), "batch_paths"), (dict(batch_paths=768), "batch_paths"),
                                    (dict(batch_paths=(1 << 24) + 512), "batch_paths"),
                                    (dict(batch_paths=-512), "batch_paths"), (dict(trace_grid=-8), "trace_grid"),
                                    (dict(trace_grid=12), "trace_grid"), (dict(dir_bins=2), "dir_bins"),
                                    (dict(dir_bins=8), "dir_bins"), (dict(dir_bins=-1), "dir_bins")])
def test_malformed_tunings(t, word):
    ok, msg = m.validate_tuning(**t)
    assert not ok and word in msg


def test_results_file_roundtrip(tmp_path):
    f = tmp_path / "tune.txt"
    assert m.tune_cache_lookup(f, "a") is None  # no file yet
    m.tune_cache_store(f, "dev=x paths=1", batch_paths=4096, trace_grid=64, dir_bins=1, ms=1.5)
    m.tune_cache_store(f, "dev=x paths=2", trace_grid=128, ms=2.25)
    assert m.tune_cache_lookup(f, "dev=x paths=1") == dict(batch_paths=4096, trace_grid=64, dir_bins=1, ms=1.5)
    assert m.tune_cache_lookup(f, "dev=x paths=2") == dict(batch_paths=0, trace_grid=128, dir_bins=0, ms=2.25)
    assert m.tune_cache_lookup(f, "dev=x paths=") is None  # keys match whole
    assert m.tune_cache_lookup(f, "dev=x paths=10") is None
    # a new result replaces the key's line and keeps the others
    m.tune_cache_store(f, "dev=x paths=1", batch_paths=8192, ms=1.25)
    lines = f.read_text().splitlines()
    assert len(lines) == 2 and sum(l.startswith("dev=x paths=1\t") for l in lines) == 1
    assert m.tune_cache_lookup(f, "dev=x paths=1") == dict(batch_paths=8192, trace_grid=0, dir_bins=0, ms=1.25)
    assert m.tune_cache_lookup(f, "dev=x paths=2")["trace_grid"] == 128
    assert not list(tmp_path.glob("*.tmp.*"))  # the temporary file was renamed over the results file


def test_damaged_lines_are_skipped(tmp_path):
    f = tmp_path / "tune.txt"
    f.write_text("k\t4096 64 1 1.0\n"        # good
                 "k\t100 64 1 0.5\n"         # batch not a multiple of 512
                 "k\t4096 12 1 0.5\n"        # grid not a multiple of 8
                 "k\t4096 64 3 0.5\n"        # bins not 0, 1, 4
                 "k\tgarbage\n"
                 "k 4096 64 1 0.5\n"         # no tab
                 "\n")
    assert m.tune_cache_lookup(f, "k") == dict(batch_paths=4096, trace_grid=64, dir_bins=1, ms=1.0)


def test_store_rejects_bad_input(tmp_path):
    f = tmp_path / "tune.txt"
    for key in ("a\tb", "a\nb", ""):
        with pytest.raises(m.SddError):
            m.tune_cache_store(f, key, ms=1.0)
    with pytest.raises(m.SddError):
        m.tune_cache_store(f, "k", batch_paths=100, ms=1.0)
    with pytest.raises(m.SddError):
        m.tune_cache_store(f, "k", ms=-1.0)
    with pytest.raises(m.SddError):
        m.tune_cache_store(tmp_path / "no_such_dir" / "t.txt", "k", ms=1.0)
    assert not f.exists()


def test_null_context_and_arguments():
    """The context entry points refuse a null context or null outputs without a device."""
    import ctypes as C
    INVALID = -1  # SDD_ERR_INVALID_ARG
    L = m.lib()
    t = m.Tuning()
    assert L.sdd_set_tuning(None, C.byref(t)) == INVALID
    assert L.sdd_get_tuning(None, C.byref(t)) == INVALID
    buf = C.create_string_buffer(64)
    assert L.sdd_tune_key(None, 1, None, buf, 64) == INVALID
    ms, fc = C.c_double(0.0), C.c_int32(0)
    assert L.sdd_autotune(None, 1, None, 1, None, C.byref(t), C.byref(ms), C.byref(fc)) == INVALID
    found = C.c_int32(0)
    assert L.sdd_tune_cache_lookup(None, b"k", C.byref(t), None, C.byref(found)) == INVALID
    assert L.sdd_tune_cache_store(b"/tmp/x", b"k", None, 1.0) == INVALID
    assert L.sdd_validate_tuning(None, None, 0) == INVALID
