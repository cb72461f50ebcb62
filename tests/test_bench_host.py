"""Host logic of the benchmark line: the algorithmic byte model of the
roofline kernel, the choice of launches a detection kernel is averaged over,
and the single-GPU guard.  No GPU is used."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stats(**kw):
    st = dict(spheres=1000, clumps=300, bins=5000, pairs=2000, upper=1800, contact_sides=3000,
              fp32=True, guard=True, learned=True, detect_fraction=0.05)
    st.update(kw)
    return st


def test_reduction_bytes_follow_the_per_unit_model():
    st = _stats()
    v = 16
    want = (1800 * (4 + 2 * v) + 2000 * 2 * v + 1000 * (20 + 4 * 0.05) + 300 * (268 + 64 + 4))
    assert bench.algorithmic_bytes("k_reduce_waves", st) == want
    # plain path: no guard words, no envelope, no margins
    st = _stats(guard=False, learned=False, detect_fraction=1.0)
    assert bench.algorithmic_bytes("k_reduce_waves", st) == 1800 * 36 + 2000 * 32 + 1000 * 20 + 300 * 268
    # FP64 contributions double the contribution vector
    st = _stats(fp32=False)
    assert bench.algorithmic_bytes("k_reduce_waves", st) - bench.algorithmic_bytes("k_reduce_waves", _stats()) \
        == 1800 * 2 * 16 + 2000 * 2 * 16


def test_pair_bytes_follow_the_per_unit_model():
    st = _stats()
    want = 2000 * (8 + 24 + 32) + 1800 * 16 + 1500 * 24 + 1000 * (8 + 16) + 300 * 128
    assert bench.algorithmic_bytes("k_pairs", st) == want


def test_detection_kernel_is_averaged_over_working_launches():
    res = dict(prof={"k_narrow": (200, 100.0), "k_pairs": (200, 50.0)}, prof_timed={}, detections=10,
               steps=200, counts=dict(pairs=2000, candidates=3800, audits=2), contact_sides=3000)
    r = bench.roofline(res, dict(spheres=1000, clumps=300, bins=5000, fp32=True), "learned")
    assert r["kernel"] == "k_narrow" and r["timed_region"] is False
    assert abs(r["avg_launch_us"] - 100.0 / 10 * 1e3) < 1e-9  # 10 detections, not 200 launches


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
