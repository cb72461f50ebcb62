"""Host logic of the benchmark line: the byte models of the roofline kernel
(the scope table's per-unit terms and the library's record layout), the
choice of launches a detection kernel is averaged over, the audit-inclusive
rate, and the single-GPU guard.  No GPU is used."""
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
    v, t = 16, 12  # force with its contact word, torque packed
    want = (1800 * (4 + v + t) + 2000 * (v + t) + 1000 * (20 + 4 * 0.05) + 300 * (268 + 64 + 4))
    assert bench.layout_bytes("k_reduce_waves", st) == want
    # plain path: no guard words, no envelope, no margins
    st = _stats(guard=False, learned=False, detect_fraction=1.0)
    assert bench.layout_bytes("k_reduce_waves", st) == 1800 * 32 + 2000 * 28 + 1000 * 20 + 300 * 268
    # FP64 contributions double both vectors
    st = _stats(fp32=False)
    assert bench.layout_bytes("k_reduce_waves", st) - bench.layout_bytes("k_reduce_waves", _stats()) \
        == 1800 * (16 + 12) + 2000 * (16 + 12)


def test_pair_bytes_follow_the_per_unit_model():
    st = _stats()
    want = 2000 * (8 + 24 + 16 + 12) + 1800 * 12 + 1500 * 24 + 1000 * (8 + 16) + 300 * 128
    assert bench.layout_bytes("k_pairs", st) == want


def test_detection_kernel_is_averaged_over_working_launches():
    res = dict(prof={"k_narrow": (200, 100.0), "k_pairs": (200, 50.0)}, prof_timed={}, detections=3,
               pass_detections=10, steps=200, counts=dict(pairs=2000, candidates=3800, audits=2),
               contact_sides=3000, audit=dict(audits=1))
    r = bench.roofline(res, dict(spheres=1000, clumps=300, bins=5000, fp32=True), "learned")
    assert r["kernel"] == "k_narrow" and r["timed_region"] is False
    assert abs(r["avg_launch_us"] - 100.0 / 10 * 1e3) < 1e-9  # 10 detections of the pass, not 200 launches


def test_survey_terms():
    """Per-sphere-step bytes as the scope table states them: B_plain = 454 +
    220 p; B_del = 234 + 148 p + 8 (p_m - p) + (244 + 72 p_m) / k; the
    reduction's a8 + a9 (+ 24 B guard) and the pair kernel's a7 per sphere."""
    assert bench.survey_step_bytes(2.5, 2.5, 1, False) == 454 + 220 * 2.5
    assert abs(bench.survey_step_bytes(2.5, 4.0, 20, True) - (234 + 148 * 2.5 + 8 * 1.5 + (244 + 72 * 4) / 20)) < 1e-12
    # the worked example of the scope table: p = 2.5, p_m = 4, k = 20 -> about 643 B
    assert abs(bench.survey_step_bytes(2.5, 4.0, 20, True) - 643) < 1
    st = _stats()  # 1000 spheres, 1500 contact pairs, 2000 candidate pairs
    p, pm = 1.5, 2.0
    assert abs(bench.survey_kernel_bytes("k_reduce_waves", st) - 1000 * (16 + 56 * p + 84 + 24)) < 1e-6
    assert abs(bench.survey_kernel_bytes("k_pairs", st) - 1000 * (60 + 92 * p + 8 * (pm - p))) < 1e-6
    assert abs(bench.survey_kernel_bytes("k_narrow", st) - 1000 * (64 + 8 * pm)) < 1e-6
    assert abs(bench.survey_kernel_bytes("k_carry", st) - 1000 * 64 * pm) < 1e-6


def test_audit_cost_is_amortised_over_its_period():
    res = dict(seconds=0.1, steps=20, audit=dict(audits=1, steps=100, chain_ms=12.0, missed=0),
               window=dict(detections=1), counts=dict(pairs=2000, candidates=3800, missed=0), contact_sides=3000,
               tune={}, graph=0, detections=1)
    line = bench.path_line(res, 1000, dict(spheres=1000, clumps=300, bins=5000, fp32=True), "learned")
    assert abs(line["sphere_steps_per_s_no_audit"] - 1000 * 20 / 0.1) < 1e-6
    assert abs(line["sphere_steps_per_s"] - 1000 * 20 / (0.1 + 20 * 0.12e-3)) < 1e-6
    assert line["k_effective"] == 20


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
