"""bench.py's accounting on the host: the cache query's algorithmic flops and
the gating of the measured HBM traffic on the kernel sources it was taken on."""
import os

import pytest

import bench


def test_query_flops_count_the_split_network():
    # per (path, wavelength): hidden layers 1..4 and the output; per path layer
    # 0's 48 position/direction inputs; per wavelength its 16 one-blob inputs
    paths, nl = 1000, 41
    rows = paths * nl
    expect = 2 * (rows * (4 * 64 * 64 + 64) + paths * 48 * 64 + nl * 16 * 64)
    assert bench.nrc_query_flops(rows, nl) == expect
    # the full network per row, minus what the split shares, is what it saves
    full = 2 * rows * (5 * 64 * 64 + 64)
    assert full - expect == 2 * (rows * 64 * 64 - paths * 48 * 64 - nl * 16 * 64)


def _write(path, sha, workload="furnished_room", grid="4x4x2"):
    with open(path, "w") as f:
        f.write("# comment=ignored\n")
        f.write(f"workload={workload}\ngrid={grid}\ndispatches=72\n")
        f.write("fetch_kib_per_dispatch=100.0\nwrite_kib_per_dispatch=50.0\n")
        f.write("fetch_scale=2.0\nwrite_scale=1.0\n")
        f.write(f"source_sha256={sha}\n")


def test_traffic_is_gated_on_sources_workload_and_grid(tmp_path, monkeypatch):
    srcs = bench.TRAFFIC["furnished_room"][1]
    f = tmp_path / "t.txt"
    monkeypatch.setitem(bench.TRAFFIC, "furnished_room", (str(f), srcs, "furnished_room"))
    _write(f, bench.source_hash(srcs))
    assert bench.measured_traffic("furnished_room", (4, 4, 2)) == (100.0 * 2.0 + 50.0) * 1024.0
    assert bench.measured_traffic("furnished_room", (2, 2, 2)) is None  # another grid
    _write(f, "0" * 64)
    assert bench.measured_traffic("furnished_room", (4, 4, 2)) is None  # other kernel sources
    _write(f, bench.source_hash(srcs), workload="nrc_room")
    assert bench.measured_traffic("furnished_room", (4, 4, 2)) is None  # another workload
    os.remove(f)
    assert bench.measured_traffic("furnished_room", (4, 4, 2)) is None  # no summary
    assert bench.measured_traffic("no_such_workload", (1, 1, 1)) is None


@pytest.mark.parametrize("key", sorted(bench.TRAFFIC))
def test_committed_traffic_summaries_parse(key):
    path, srcs, workload = bench.TRAFFIC[key]
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.lstrip().startswith("#"))
    assert kv["workload"] == workload
    for k in ("fetch_kib_per_dispatch", "write_kib_per_dispatch", "fetch_scale", "write_scale"):
        assert float(kv[k]) > 0
    assert len(kv["source_sha256"]) == 64


def test_relmse_fit_and_frames_to_target():
    n = [(k, 0.1 * k, 0.004 + 40.0 / k) for k in range(100, 401, 10)]
    a, b = bench.relmse_fit(n, floor=True)
    assert abs(a - 0.004) < 1e-12 and abs(b - 40.0) < 1e-9
    a0, b0 = bench.relmse_fit([(k, 0.0, 40.0 / k) for k in range(1, 50)], floor=False)
    assert a0 == 0.0 and abs(b0 - 40.0) < 1e-9
    assert abs(bench.frames_to(0.01, 0.004, 40.0) - 40.0 / 0.006) < 1e-9
    assert bench.frames_to(0.01, 0.01, 40.0) is None and bench.frames_to(0.01, 0.02, 40.0) is None


def test_error_split_recovers_bias_and_variance():
    """Synthetic images: truth T, reference halves with noise s_r, a test image
    whose halves carry noise s_i and a known bias; the split recovers the
    weighted squared bias and variance within its own standard error."""
    import torch
    g = torch.Generator().manual_seed(3)
    P, L = 200_000, 4
    T = 0.5 + torch.rand(P, L, generator=g, dtype=torch.float64)
    bias = 0.05 * T
    s_r, s_i = 0.3, 0.2
    R1 = T + s_r * torch.randn(P, L, generator=g, dtype=torch.float64)
    R2 = T + s_r * torch.randn(P, L, generator=g, dtype=torch.float64)
    R, varR = 0.5 * (R1 + R2), 0.25 * (R1 - R2) ** 2
    Ia = T + bias + s_i * torch.randn(P, L, generator=g, dtype=torch.float64)
    Ib = T + bias + s_i * torch.randn(P, L, generator=g, dtype=torch.float64)
    w = 1.0 / T ** 2
    b2, se, var_w = bench.error_split(Ia, Ib, R, varR, w)
    want = float((bias ** 2 * w).mean())
    assert abs(b2 - want) <= 4 * se, (b2, want, se)
    assert abs(var_w - float((s_i ** 2 / 2 * w).mean())) <= 0.02 * var_w
    # an unbiased image: the split's bias is zero within its error
    b0, se0, _ = bench.error_split(Ia - bias, Ib - bias, R, varR, w)
    assert abs(b0) <= 4 * se0
