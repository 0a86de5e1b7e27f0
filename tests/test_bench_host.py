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
        ("at::native::elementwise_kernel<...>", "FETCH_SIZE", 7.0),  # every kernel is kept, by full name
    ]
    with open(tmp_path / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i, k, c, v])
    got = bench._counter_means(str(tmp_path), "FETCH_SIZE")
    assert got == {"ptd::fused::k_fused_fwd<double, Shape<...>>(...)": 200.0,
                   "ptd::(anonymous namespace)::k_copy16(...)": 50.0, "at::native::elementwise_kernel<...>": 7.0}


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
    k14 = "void ptd::fused::k_fused_fwd<double, ptd::fused::Shape<double, 14, 9, 512, 3>, false, 3>(x)"
    k13 = "void ptd::fused::k_fused_fwd<double, ptd::fused::Shape<double, 13, 9, 512, 3>, true, 3>(x)"
    rec = {"kernel_hash": bench._kernel_hash(),
           "kernels": {k14: {"fetch_bytes": 100, "write_bytes": 23}, k13: {"fetch_bytes": 1, "write_bytes": 2}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench._traffic_total("k_fused_fwd<double", "Shape<double, 14,", ", false,") == 123
    assert bench._traffic_total("k_fused_fwd<double", "Shape<double, 13,", ", true,") == 3
    assert bench._traffic_total("k_fused_fwd<double") is None  # two kernels match: ambiguous
    assert bench._traffic_total("k_fused_fwd<double", "Shape<double, 12,") is None
    (csrc / "k.hip").write_text("v2")
    assert bench._traffic_total("k_fused_fwd<double", "Shape<double, 14,", ", false,") is None


def test_write_traffic_scales_every_kernel_by_the_copy(bench, tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every kernel, scaled so
    that the reference copy reads and writes the matrix once each."""
    import json

    csrc = tmp_path / "paper_2403_11644_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("v1")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    n = 4
    mat_kib = 16 * 4 ** n / 1024.0
    rows = {"f": [("ptd::k_copy16(a)", mat_kib / 2), ("ptd::k_x<float>(b)", mat_kib), ("at::other(c)", 1.0)],
            "w": [("ptd::k_copy16(a)", mat_kib), ("ptd::k_x<float>(b)", 3 * mat_kib), ("at::other(c)", 1.0)]}
    for d, counter in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        (tmp_path / d).mkdir()
        lines = ["Kernel_Name,Counter_Name,Counter_Value"]
        lines += ['"%s",%s,%r' % (k, counter, v) for k, v in rows[d]]
        (tmp_path / d / "p_counter_collection.csv").write_text("\n".join(lines) + "\n")
    data = bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), n)
    assert data["fetch_scale"] == 2.0 and data["write_scale"] == 1.0
    assert "at::other(c)" not in data["kernels"]  # the library's kernels only
    assert data["kernels"]["ptd::k_x<float>(b)"] == {"fetch_bytes": 2 * 16 * 4 ** n, "write_bytes": 3 * 16 * 4 ** n}
    assert json.loads((tmp_path / "profiles" / "traffic.json").read_text()) == data
    assert bench._traffic("k_x<float>") == (2 * 16 * 4 ** n, 3 * 16 * 4 ** n)


def test_counter_means_merge_every_file_of_a_folder(bench, tmp_path):
    # a second counter pass over other legs writes into the same folder under
    # another prefix: both files are read, and a kernel seen in both is
    # averaged over all its dispatches
    def write(name, rows):
        with open(tmp_path / name, "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
            for r in rows:
                w.writerow(r)
    write("f_counter_collection.csv", [("k_a(...)", "FETCH_SIZE", 10.0), ("k_both(...)", "FETCH_SIZE", 2.0)])
    write("fb_counter_collection.csv", [("k_b(...)", "FETCH_SIZE", 30.0), ("k_both(...)", "FETCH_SIZE", 4.0),
                                        ("k_both(...)", "FETCH_SIZE", 6.0)])
    m = bench._counter_means(str(tmp_path), "FETCH_SIZE")
    assert m == {"k_a(...)": 10.0, "k_b(...)": 30.0, "k_both(...)": 4.0}
