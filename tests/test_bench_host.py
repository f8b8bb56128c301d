"""Host logic of bench.py on the CPU: the recorded HBM traffic is reported
only for the kernel source, precision, width and tile it was measured on,
and a multi-GPU request is refused."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_record_follows_the_kernel_source():
    """The recorded bytes are reported while the kernel's sources have the
    recorded SHA-1, and null once they have changed."""
    import hashlib
    bench = _bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    got = bench.measured_traffic(rec["dtype"], rec["rhs"], rec.get("tn"))
    h = hashlib.sha1()
    for rel in rec["sources"]:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    if h.hexdigest() == rec["sources_sha1"]:
        assert got == rec["traffic_bytes_per_launch"] and got > 0
    else:
        assert got is None


def test_traffic_is_null_for_another_configuration():
    bench = _bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    other = "f64" if rec["dtype"] == "f32" else "f32"
    assert bench.measured_traffic(other, rec["rhs"], rec.get("tn")) is None
    assert bench.measured_traffic(rec["dtype"], rec["rhs"] + 1, rec.get("tn")) is None
    assert bench.measured_traffic(rec["dtype"], rec["rhs"], 999) is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout
