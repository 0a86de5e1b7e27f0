"""Host logic of bench.py, without a GPU: the one-GPU guard, the counter
summary that turns rocprofv3 --pmc folders into bytes per launch, the
Hermitian byte count, the kernel-sources hash, and the stale-record rule of
the traffic lookup."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as B

    return B


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_means(bench, tmp_path):
    rows = [
        ("ptd::fused::k_fused_fwd<double, Shape<...>>(...)", "FETCH_SIZE", 100.0),
        ("ptd::fused::k_fused_fwd<double, Shape<...>>(...)", "FETCH_SIZE", 300.0),
        ("ptd::(anonymous namespace)::k_copy16(...)", "FETCH_SIZE", 50.0),
        ("ptd::(anonymous namespace)::k_copy16(...)", "WRITE_SIZE", 999.0),  # other counter: ignored
        ("at::native::elementwise_kernel<...>", "FETCH_SIZE", 7.0),  # other kernel: ignored
    ]
    with open(tmp_path / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i, k, c, v])
    got = bench._counter_means(str(tmp_path), "FETCH_SIZE")
    assert got == {"k_fused_fwd": 200.0, "k_copy16": 50.0}


def test_hermitian_bytes(bench):
    # n >= 5: half of A (mirrored pairs read once) plus the real output
    assert bench._herm_bytes(13, 16) == 4.0 ** 13 * (8 + 8)
    # n <= 4: all of A plus the real output
    assert bench._herm_bytes(3, 8) == 64 * (8 + 4)


def test_kernel_hash_covers_device_sources_only(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2403_11644_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("kernel A")
    (csrc / "b.hpp").write_text("header B")
    (csrc / "host.cpp").write_text("host code")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench._kernel_hash()
    (csrc / "host.cpp").write_text("host code, changed")
    assert bench._kernel_hash() == h0
    (csrc / "b.hpp").write_text("header B, changed")
    assert bench._kernel_hash() != h0


def test_traffic_record_is_dropped_once_the_sources_change(bench, tmp_path, monkeypatch):
    import json

    csrc = tmp_path / "paper_2403_11644_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("v1")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"k_fused_fwd/n14/c128": {"kernel_hash": bench._kernel_hash(), "bytes_per_launch": 123.0}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench._traffic("k_fused_fwd", "n14/c128") == 123.0
    assert bench._traffic("k_fused_fwd", "n13/c128") is None
    (csrc / "k.hip").write_text("v2")
    assert bench._traffic("k_fused_fwd", "n14/c128") is None
