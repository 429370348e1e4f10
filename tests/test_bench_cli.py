"""Host-side checks of the benchmark's command line and of its measured-traffic
table (no GPU): the run refuses more than one GPU, and the per-launch bytes it
reports are keyed by a digest of the kernel sources, so that they read null
once the kernels change."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_traffic_keyed_by_kernel_sources(bench, monkeypatch):
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    key = "shear64_v32_nh1_kn1_st1/fp64/update_int"
    if h.hexdigest()[:16] == bench.MEASURED_TRAFFIC["sources_sha256_16"]:
        assert bench.traffic_bytes("shear64_v32_nh1_kn1_st1", "fp64", "update_int") == \
            bench.MEASURED_TRAFFIC["bytes"][key]
    # any other digest: the bytes are not reported
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256_16", "0" * 16)
    assert bench.traffic_bytes("shear64_v32_nh1_kn1_st1", "fp64", "update_int") is None
