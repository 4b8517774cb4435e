"""The benchmark's command line (CPU): more than one GPU is refused with a
message before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_lists_its_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for w in ("lognormal129", "lognormal257", "batched129", "sphere97"):
        assert w in r.stdout


def test_traffic_is_read_only_for_the_launch_shape_it_was_taken_on():
    """The HBM traffic in the bench line comes from a committed counter summary
    of the same kernel source and launch shape; any other shape reports null."""
    sys.path.insert(0, ROOT)
    import bench
    on_file = {(768, 11, 2, 1), (1024, 17, 2, 1), (512, 17, 2, 1)}
    for t, r, nb, band in on_file:
        b = bench.read_traffic("lognormal129", {"threads": t, "rays": r, "bundles": nb, "band": band})
        assert b is not None and 5e10 < b < 1e12
    assert bench.read_traffic("lognormal129", {"threads": 768, "rays": 11, "bundles": 2, "band": 0}) is None
    assert bench.read_traffic("lognormal129", {"threads": 512, "rays": 9, "bundles": 4, "band": 1}) is None
    assert bench.read_traffic("no_such_workload", {"threads": 768, "rays": 11, "bundles": 2, "band": 1}) is None
