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
    monkeypatch.setitem(bench.TRAFFIC, "furnished_room", (str(f), srcs))
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


@pytest.mark.parametrize("workload", sorted(bench.TRAFFIC))
def test_committed_traffic_summaries_parse(workload):
    path, srcs = bench.TRAFFIC[workload]
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.lstrip().startswith("#"))
    assert kv["workload"] == workload
    for k in ("fetch_kib_per_dispatch", "write_kib_per_dispatch", "fetch_scale", "write_scale"):
        assert float(kv[k]) > 0
    assert len(kv["source_sha256"]) == 64
