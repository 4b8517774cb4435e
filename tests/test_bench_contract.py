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


def test_traffic_is_read_only_for_the_launch_shape_it_was_taken_on(tmp_path):
    """The HBM traffic in the bench line comes from a counter summary of the
    same kernel source and launch shape; any other shape, workload or kernel
    source reports null."""
    sys.path.insert(0, ROOT)
    import bench
    src = bench.fs_source_hash()
    for name, shape, hbm, h in (("a", "768,11,2,band", 1.08e11, src), ("b", "1024,17,2,band", 2.77e11, src),
                                ("c", "512,9,4,band", 3.0e11, "0123456789abcdef")):
        (tmp_path / f"fs_box_lognormal129_traffic_{name}.md").write_text(
            f"fs_box.hip sha256[:16]: {h}\nhbm_bytes_per_launch: {hbm:e}\nlaunch_shape: {shape}\n")
    rd = lambda w, t, r, nb, band: bench.read_traffic(w, {"threads": t, "rays": r, "bundles": nb, "band": band},
                                                      str(tmp_path))  # noqa: E731
    assert rd("lognormal129", 768, 11, 2, 1) == 1.08e11
    assert rd("lognormal129", 1024, 17, 2, 1) == 2.77e11
    assert rd("lognormal129", 768, 11, 2, 0) is None      # other tile kind
    assert rd("lognormal129", 512, 9, 4, 1) is None       # taken on another kernel source
    assert rd("no_such_workload", 768, 11, 2, 1) is None
