"""Throughput of the clumped-sphere DEM timestep on one MI355X.

Workload (default): the rover-scale bed, ~11M clumps / ~34M spheres of the
eight bed templates tiled from a patch settled on the GPU, with a
20,000-sphere wheel driven at slip 0.2; FP32 force arithmetic, FP64 state and
history.  One step = pose, detection (every step in plain mode, when due in
deferred modes), Hertz-Mindlin force with tangential history, reduction onto
clumps and integration.

Prints one JSON line: sphere-timesteps/s of the deferred-detection path (the
value), the plain per-step-detection path beside it, a roofline entry for the
dominant kernel (HIP-event durations inside the timed region) and the FP64
CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the kernel with the largest share of a learned-interval step, timed with HIP
# events inside the timed region
ROOFLINE_KERNEL = "k_reduce_waves"
# detection settings of the timed deferred paths (FP32 force arithmetic)
DETECT = dict(k_max=20, safety=1.5, margin_cap=2e-4, audit_period=100)
METRIC = "sphere-timesteps/s at 34M spheres, learned-CD vs plain, 0 missed contacts"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- byte models
def algorithmic_bytes(kernel: str, st: dict) -> float:
    """Bytes a launch of `kernel` must move at minimum: every array it reads or
    writes touched once (gathers of neighbour data counted as cache hits).
    P pairs of the active set, U of them sphere pairs (each also listed in the
    higher sphere's upper segment), C contact pairs, v one contribution vector
    (force or torque with a fourth word: float4 or double4)."""
    ns, nc, cells = st["spheres"], st["clumps"], st["bins"]
    P, U, C = st["pairs"], st["upper"], st["contact_sides"] / 2.0
    v = 16 if st["fp32"] else 32
    mat = 16 if st["fp32"] else 32
    guard, learned = st["guard"], st.get("learned", False)
    det_frac = st.get("detect_fraction", 1.0)  # share of the launches on a step with a detection
    if kernel == "k_pose":
        # per sphere: owner, template sphere, position write (+ speed), scene
        # and bin write (the count's atomic); per clump its record
        return ns * (8 + 32 + (4 if guard else 0) + 8) + nc * 128
    if kernel == "k_cell_count":
        return ns * 48
    if kernel == "k_cell_scatter":
        return ns * 132
    if kernel == "k_narrow":
        # positions, margins, bin starts; new pairs (partner, own id, history),
        # upper entries (partner, own id), the current pairs merged for history
        return ns * 88 + cells * 8 + 32 * P + 8 * U + 28 * P
    if kernel == "k_link":
        return U * 28
    if kernel == "k_pairs":
        # per pair: own id, partner, history read, force and torque of the lower
        # sphere; per sphere pair the partner's torque; per contact the history
        # write; compulsory per-sphere and per-clump gathers (owner, template
        # sphere, material; the clump record)
        return P * (8 + 24 + 2 * v) + U * v + C * 24 + ns * (8 + mat) + nc * 128
    if kernel == "k_reduce_waves":
        # per upper entry: link, the pair's force and the partner's torque; per
        # pair: force and torque of the lower sphere; per sphere: clump position
        # and segment bounds (+ margin for the guard on a detection's step:
        # later steps test a per-clump bound first); per clump: record read and
        # write, template, scene, prescribed-motion index (+ its pose at the last
        # detection for the guard, + acceleration envelope when learned)
        return (U * (4 + 2 * v) + P * 2 * v + ns * (20 + (4 * det_frac if guard else 0)) +
                nc * (268 + (64 if guard else 0) + (4 if learned else 0)))
    if kernel in ("k_scan_reduce", "k_scan_final"):
        return cells * (4 if kernel == "k_scan_reduce" else 8)
    if kernel == "k_detect_begin":
        return cells * 8
    return 0.0


def make_scene(desc, mode, mlp=None):
    """The scene as the benchmark times it: FP32 force arithmetic, detection `mode`."""
    from paper_2307_03445_amd._lib import Scene
    sc = Scene(desc, precision="fp32")
    if mode == "learned":
        sc.set_mlp(mlp)
    if mode != "plain":
        sc.set_detection(mode, **DETECT)
    return sc


def run_path(desc, mode, steps, warmup, mlp=None):
    import torch
    audit_every = DETECT["audit_period"]
    sc = make_scene(desc, mode, mlp)
    t0 = time.perf_counter()
    sc.step(warmup)
    # bin size and launch shape from the library's autotuner (its trials are
    # ordinary steps, each of one detection and the steps up to the next at
    # the interval bound), then steps to settle before timing
    tune = sc.autotune(DETECT["k_max"])
    sc.step(warmup)
    log(f"[{mode}] warmup {2 * warmup} steps and autotuning ({tune}): {time.perf_counter() - t0:.2f} s")
    c0 = sc.counts()
    # Inside the timed region only the kernel the roofline is quoted for is
    # bracketed by events (events around every kernel cost about 5 % of a
    # step); the per-kernel table comes from a short pass afterwards.
    sc.profile(True, only=(ROOFLINE_KERNEL,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    from paper_2307_03445_amd._lib import CdemError
    done = 0
    while done < steps:
        n = min(audit_every, steps - done) if mode != "plain" else steps - done
        try:
            sc.step(n)
        except CdemError as e:  # an audit found a missed contact: the steps still ran; report it
            if e.code != -5:
                raise
            log(f"[{mode}] audit reported missed contacts: {e}")
        done += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof_timed = sc.profile_read()
    c1 = sc.counts()
    contact_sides = sc.last_step_contacts()
    # every kernel, over one audit period more (not timed)
    sc.profile(True)
    try:
        sc.step(min(audit_every, steps) if mode != "plain" else min(20, steps))
    except CdemError as e:
        if e.code != -5:
            raise
    prof = sc.profile_read()
    sc.profile(False)
    sc.close()
    dets = c1["detections"] - c0["detections"]
    log(f"[{mode}] {steps} steps in {dt:.3f} s; detections {dets}; candidates {c1['candidates']}; "
        f"contact sides {contact_sides}")
    for k, (n, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"    {k:22s} launches {n:6d} total {ms:9.2f} ms  avg {ms / n * 1e3:9.1f} us")
    return dict(seconds=dt, prof=prof, prof_timed=prof_timed, counts=c1, detections=dets,
                contact_sides=contact_sides, guard_trips=c1["guard_trips"] - c0["guard_trips"], tune=tune,
                steps=steps)


KERNEL_SOURCES = ("paper_2307_03445_amd/csrc/kernels.hip", "paper_2307_03445_amd/csrc/cdem_internal.h",
                  "paper_2307_03445_amd/csrc/mlp_dev.h")
COUNTERS = os.path.join(ROOT, "profiles", "counters_rover_bed.json")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a device copy of known size), or None when there is no
    summary for it or the kernels changed since it was taken."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != kernel_source_hash() or kernel not in c.get("kernels", {}):
        return None
    k = c["kernels"][kernel]
    return 1024.0 * (k["fetch_kib"] * c["fetch_scale"] + k["write_kib"] * c["write_scale"])


def roofline(res, desc_stats, mode):
    # dominant kernel from the full per-kernel pass; its time from the timed
    # region when it is the one timed there
    prof = res["prof"]
    k, (n, ms) = max(prof.items(), key=lambda kv: kv[1][1])
    timed = k in res["prof_timed"]
    if timed:
        n, ms = res["prof_timed"][k]
    cnt = res["counts"]
    st = dict(desc_stats, pairs=cnt["pairs"], upper=cnt["candidates"] - cnt["pairs"],
              contact_sides=res["contact_sides"], guard=(mode != "plain"), learned=(mode == "learned"),
              detect_fraction=min(1.0, res["detections"] / max(1, res["steps"])))
    # a detection kernel early-exits when no detection is due: count only real launches
    launches = n
    if k == "k_pose":  # works on the steps that detect or audit
        launches = max(1, res["detections"] + res["counts"].get("audits", 0))
    if k in ("k_narrow", "k_link", "k_cell_count", "k_cell_scatter", "k_detect_begin", "k_scan_reduce",
             "k_scan_final"):
        launches = max(1, res["detections"])
    b = algorithmic_bytes(k, st)
    avg_s = ms / 1e3 / launches
    gbs = b / avg_s / 1e9 if b else None
    return dict(bound="hbm", kernel=k, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(gbs / HBM_PEAK_GBS) if gbs else None, traffic=measured_traffic(k),
                bytes_per_launch=b, avg_launch_us=avg_s * 1e6, timed_region=timed)


def cpu_baseline(seconds_target=15.0):
    import oracle
    from paper_2307_03445_amd import inputs as I
    oracle.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(cores)
    d = I.walled_box()
    o = oracle.Oracle(d)
    o.step(5)
    t0 = time.perf_counter()
    o.step(20)
    per = (time.perf_counter() - t0) / 20
    n = int(max(20, min(20000, seconds_target / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return dict(value=d.n_spheres * n / dt, unit="sphere-timesteps/s", cores=cores, kind="oracle",
                sample=f"walled box (2,000 three-sphere clumps, 6,000 spheres, lattice in a walled box), "
                       f"{n} steps of FP64 O(N^2) brute force, {dt:.1f} s")


def gpu_on_cpu_sample(steps=2000):
    """The GPU on the oracle's own sample: the walled box in the all-FP64 mode
    with per-step detection (6,000 spheres: a launch-bound size, far below
    what fills the chip), for a like-for-like rate beside the oracle's."""
    import torch
    from paper_2307_03445_amd import inputs as I
    from paper_2307_03445_amd._lib import Scene
    sc = Scene(I.walled_box(), precision="fp64")
    sc.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ns = sc.counts()["spheres"]
    sc.close()
    return dict(value=ns * steps / dt, unit="sphere-timesteps/s", precision="fp64", detection="plain",
                sample=f"walled box, {steps} steps (launch-bound at 6,000 spheres)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--clumps", type=int, default=11_000_000)
    ap.add_argument("--modes", default="plain,fixed,learned")
    ap.add_argument("--mlp", default=None, help="npz with envelope-MLP parameters (default: the package's "
                                                "trained weights, else train now)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--patch-cache", default=None,
                    help="npz file holding the settled preparation patch (written if missing)")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (counter calibration)")
    ap.add_argument("--copy-bandwidth-gib", type=float, default=0.0,
                    help="only time device-to-device copies of this many GiB (achievable HBM bandwidth)")
    args = ap.parse_args()
    if args.copy_bandwidth_gib > 0:
        import torch
        n = int(args.copy_bandwidth_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        print(json.dumps({"copy_bytes_read_and_written": 8 * n, "seconds_per_copy": sec,
                          "GB_per_s": 8 * n / sec / 1e9, "copies_timed": reps}))
        return
    if args.copy_probe_gib > 0:
        import torch
        n = int(args.copy_probe_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this build is single-GPU).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_03445_amd import inputs as I
    from paper_2307_03445_amd import prep
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if args.patch_cache and os.path.exists(args.patch_cache):
        z = np.load(args.patch_cache)
        px, pq = z["x"], z["q"]
        log(f"patch loaded from {args.patch_cache}")
    else:
        px, pq, info = prep.settle_patch(log=log)
        log(f"patch settled: {info}")
        if args.patch_cache:
            np.savez(args.patch_cache, x=px, q=pq)
    desc = I.rover_bed(px, pq, n_clumps=args.clumps)
    log(f"workload: {desc.n_clumps} clumps, {desc.n_spheres} spheres, built in {time.perf_counter() - t0:.1f} s")
    stats = dict(spheres=desc.n_spheres, clumps=desc.n_clumps, fp32=True)
    modes = args.modes.split(",")
    mlp, mlp_info = None, None
    if "learned" in modes:
        from paper_2307_03445_amd import train
        path = args.mlp or train.WEIGHTS
        if os.path.exists(path):
            mlp = np.load(path)["params"].astype(np.float32)
            mlp_info = f"loaded {os.path.relpath(path, ROOT)}"
        else:
            t1 = time.perf_counter()
            mlp, info = train.train(px, pq, log=log)
            mlp_info = f"trained now in {time.perf_counter() - t1:.1f} s: {info}"
        log(f"envelope MLP: {mlp_info}")
    results = {}
    for mode in modes:
        r = run_path(desc, mode, args.steps, args.warmup, mlp=mlp)
        results[mode] = r
    from paper_2307_03445_amd._lib import Scene  # noqa: F401  (native library is the path)
    main_mode = "learned" if "learned" in results else ("fixed" if "fixed" in results else "plain")
    r = results[main_mode]
    sps = desc.n_spheres * args.steps / r["seconds"]
    # bins: same grid for every mode up to the margin cap; read from counts
    stats["bins"] = r["counts"]["bins"]
    line = {
        "metric": METRIC,
        "value": sps,
        "unit": "sphere-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 force / f64 state",
        "data": "synthetic",
        "config": {"workload": f"rover-scale bed: {desc.n_clumps} clumps, {desc.n_spheres} spheres "
                               f"(8 templates of 1-6 spheres, tiled from a GPU-settled patch), 20k-sphere wheel "
                               f"at slip 0.2, h=1e-6 s", "detection": main_mode},
        "paths": {m: {"sphere_steps_per_s": desc.n_spheres * args.steps / v["seconds"],
                      "ms_per_step": v["seconds"] / args.steps * 1e3, "detections": v["detections"],
                      "guard_trips": v["guard_trips"], "candidates": v["counts"]["candidates"],
                      "contact_sides": v["contact_sides"], "missed": v["counts"]["missed"],
                      "autotune": v["tune"]}
                  for m, v in results.items()},
        "envelope_mlp": mlp_info,
        "roofline": roofline(r, stats, main_mode),
    }
    if "plain" in results and main_mode != "plain":
        line["speedup_vs_plain"] = results["plain"]["seconds"] / r["seconds"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
        line["gpu_on_cpu_sample"] = gpu_on_cpu_sample()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
