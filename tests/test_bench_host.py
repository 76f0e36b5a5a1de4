"""bench.py's host-side contract, without a GPU: more than one GPU is refused
with a message and exit status 2 (the measurement is of one GPU), and the
counter traffic is reported only for the kernel sources it was taken from."""
import json
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr


def test_traffic_only_for_matching_sources(monkeypatch):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    heads = {"z_contig", "y_strided", "x_strided"}   # the headline transform's passes
    assert heads <= set(t["kernels"])
    for name in heads:   # counter bytes near the algorithmic 2 GiB per pass
        assert 0.99 < t["kernels"][name]["hbm_bytes_per_launch"] / 2 ** 31 < 1.05
    for name, k in t["kernels"].items():   # other workloads' kernels: per-dispatch bytes
        if k.get("alg_bytes_per_launch"):
            assert 0.99 < k["hbm_bytes_per_launch"] / k["alg_bytes_per_launch"] < 1.5, name
    monkeypatch.setattr(bench, "csrc_hash", lambda: t["csrc_hash"])
    assert bench.load_traffic("y_strided", 2 ** 31) == t["kernels"]["y_strided"]["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "csrc_hash", lambda: "0" * 16)
    assert bench.load_traffic("y_strided", 2 ** 31) is None
