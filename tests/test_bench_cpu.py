"""bench.py contract checks that need no GPU: a multi-GPU request exits with a message (this
build measures one GPU), and the measured-traffic figure is withheld when the rasterizer
source does not hash to the one the counters were taken with."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_profiled_kernel():
    b = _bench()

    class A:
        precision, splits, group, scene = "fp16", 2, 1, "clustered1m"
    t = b.raster_traffic(A)
    c = b.RASTER_COUNTERS
    if b.raster_source_hash() == c["sha256"]:
        assert t == 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])
    else:
        assert t is None
    A.group = 4
    assert b.raster_traffic(A) is None
    A.group, A.scene = 1, "dense6m"
    assert b.raster_traffic(A) is None
