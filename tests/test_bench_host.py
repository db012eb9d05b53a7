"""Host logic of bench.py, on the CPU: the one-GPU contract and the gate
that reports the rocprofv3 byte counts only for the kernel sources they
were taken on."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", str(n)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == n
    assert "one GPU" in line["error"]


def _fake_root(tmp_path, bench):
    for p in bench.KERNEL_SOURCES:
        dst = tmp_path / p
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, p), dst)
    (tmp_path / "profiles").mkdir()
    return tmp_path


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    import bench
    root = _fake_root(tmp_path, bench)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("f64") is None  # no summary
    summary = {"kernel_hash": bench.kernel_hash(),
               "per_launch_bytes": {"f64": 4.2e10, "f16": 1.1e10}}
    (root / "profiles" / "traffic.json").write_text(json.dumps(summary))
    assert bench.measured_traffic("f64") == 4.2e10
    assert bench.measured_traffic("f16") == 1.1e10
    assert bench.measured_traffic("f32") is None  # not profiled
    # any edit of a kernel source voids the counts
    src = root / bench.KERNEL_SOURCES[0]
    src.write_text(src.read_text() + "\n// edited\n")
    assert bench.measured_traffic("f64") is None


def test_committed_traffic_summary_is_consistent():
    """The committed summary covers every storage form, and its byte
    counts lie near the algorithmic 2 x 81 x S bytes per site of the
    256^3 vortex (the counters' calibration factors are stated in it)."""
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    assert len(t["kernel_hash"]) == 16
    sites = 2 * 256 ** 3
    for st, nbytes in bench.STORAGE_BYTES.items():
        alg = 2 * 81 * nbytes * sites
        got = t["per_launch_bytes"][st]
        assert 0.99 < got / alg < 1.05, (st, got / alg)
        for parity in ("even", "odd"):
            d = t["detail"][st][parity]
            assert 0.99 < d["read_over_alg"] < 1.05
            assert 0.99 < d["write_over_alg"] < 1.05


def test_mach_option_only_for_the_vortex():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--workload", "shear512", "--ma", "0.1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--ma applies to the tgv256 workload" in r.stderr
