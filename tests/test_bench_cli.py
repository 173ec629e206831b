"""bench.py's contract on the host: one GPU only (N > 1 exits with a
message), and the counter traffic is reported only for the kernel source it
was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_measured_kernel():
    """The table answers only for the sources it was measured on (their
    sha256), the retained-match count and the tile shape."""
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    t = bench.PMC_TRAFFIC
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    Z = next(iter(t["bytes_per_launch"]))
    tile = next(iter(t["bytes_per_launch"][Z]))
    saved = t["sources_sha256"]
    try:
        t["sources_sha256"] = h.hexdigest()
        assert bench.measured_traffic(tile, Z) == t["bytes_per_launch"][Z][tile]
        assert bench.measured_traffic(tile, Z + 1) is None
        assert bench.measured_traffic("3x5", Z) is None
        t["sources_sha256"] = "0" * 64
        assert bench.measured_traffic(tile, Z) is None
    finally:
        t["sources_sha256"] = saved
    json.dumps(t)
