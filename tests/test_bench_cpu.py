"""bench.py on the host: the one-GPU contract, the rule that HBM traffic is
reported only from counters taken on the current kernel source, and the
arithmetic of the committed counter records (bytes = counter KiB x the copy
kernel's calibration factor; algorithmic bytes = one read and one write of
every population of every node)."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

B = {"rD2Q25": 25, "rD3Q53": 53}
NODES = {"4096x4096": 4096 * 4096, "256x256x256": 256 ** 3}


@pytest.mark.parametrize("n", ["2", "8", "0"])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _records():
    d = os.path.join(ROOT, "profiles")
    return sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith("_traffic.json"))


def test_there_are_traffic_records():
    assert len(_records()) >= 4


@pytest.mark.parametrize("path", _records(), ids=os.path.basename)
def test_traffic_record_arithmetic(path):
    with open(path) as fh:
        rec = json.load(fh)
    cal = rec["calibration"]
    ff = cal["true_kib_each_way"] / cal["fetch_size_kib"]
    fw = cal["true_kib_each_way"] / cal["write_size_kib"]
    assert abs(ff - cal["fetch_factor"]) < 1e-4 and abs(fw - cal["write_factor"]) < 1e-4
    # every KiB figure is stored rounded to 0.1 KiB (relative 1e-7 at these sizes)
    rb = rec["fetch_size_kib_per_dispatch"] * ff * 1024
    wb = rec["write_size_kib_per_dispatch"] * fw * 1024
    assert abs(rec["read_bytes_per_launch"] - rb) <= 2e-7 * rb
    assert abs(rec["write_bytes_per_launch"] - wb) <= 2e-7 * wb
    total = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert abs(rec["bytes_per_launch"] - total) <= 1
    name = os.path.basename(path)[len("k_step_"):-len("_traffic.json")]
    kind, rest = name.split("_", 1)
    storage, shape = rest.rsplit("_", 1)
    assert rec["storage"] == storage and shape in rec["workload"] and kind in rec["workload"]
    alg = 2 * B[kind] * bench.STORE_BYTES[storage] * NODES[shape]
    assert rec["algorithmic_bytes_per_launch"] == alg
    assert abs(rec["traffic_over_algorithmic"] - rec["bytes_per_launch"] / alg) < 1e-4
    # the commands run committed files only
    for c in rec["commands"]:
        assert c.startswith("rocprofv3 --pmc ") and " -- python3 bench.py " in c and "_work" not in c


def _write(tmp_path, h):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    rec = {"source_hash": h, "bytes_per_launch": 123456}
    (tmp_path / "profiles" / "k_step_rD2Q25_fp32_4096x4096_traffic.json").write_text(json.dumps(rec))


def test_traffic_only_from_current_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "00aa11bb22cc33dd")
    assert bench.measured_traffic("rD2Q25", "fp32", "4096x4096", 1) is None       # no record
    _write(tmp_path, "ffffffffffffffff")
    assert bench.measured_traffic("rD2Q25", "fp32", "4096x4096", 1) is None       # stale record
    _write(tmp_path, "00aa11bb22cc33dd")
    assert bench.measured_traffic("rD2Q25", "fp32", "4096x4096", 1) == 123456
    assert bench.measured_traffic("rD2Q25", "fp64", "4096x4096", 1) is None


def test_source_hash_covers_the_kernel_sources(tmp_path, monkeypatch):
    """A change to any kernel header or to the ABI source changes the hash."""
    src = os.path.join(ROOT, "paper_2512_16230_amd", "csrc")
    names = ("device.h", "kernels.h", "lattices.h", "launch.h", "launchers.h", "mfma.h", "mfma_layout.h", "abi.hip")
    pkg = tmp_path / "paper_2512_16230_amd" / "csrc"
    pkg.mkdir(parents=True)
    for n in names:
        (pkg / n).write_bytes(open(os.path.join(src, n), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    for n in names:
        p = pkg / n
        orig = p.read_bytes()
        p.write_bytes(orig + b"\n")
        assert bench.kernel_source_hash() != h0, n
        p.write_bytes(orig)
    assert bench.kernel_source_hash() == h0
