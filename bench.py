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
import dataclasses
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
def layout_bytes(kernel: str, st: dict) -> float:
    """Bytes a launch of `kernel` moves with this library's own record layout:
    every array it reads or writes touched once (gathers of neighbour data
    counted as cache hits).  P pairs of the active set, U of them sphere
    pairs (each also listed in the higher sphere's upper segment), C contact
    pairs, v one force contribution (with a fourth word, the contact flag:
    float4 or double4), t one torque contribution (three floats or doubles)."""
    ns, nc, cells = st["spheres"], st["clumps"], st["bins"]
    P, U, C = st["pairs"], st["upper"], st["contact_sides"] / 2.0
    v = 16 if st["fp32"] else 32
    t = 12 if st["fp32"] else 24
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
        # first pass: positions, margins, bin starts; the staged counts and
        # candidates (both sides of every pair)
        return ns * 88 + cells * 8 + ns * 8 + 4 * (P + U)
    if kernel == "k_narrow_rows":
        # staged counts and candidates read; segment bounds; new pairs and
        # upper entries (partner, own id)
        return ns * 8 + 4 * (P + U) + ns * 16 + 8 * P + 8 * U
    if kernel == "k_carry":
        # new pairs' ids, the current set's bounds and partners, history read
        # and written
        return 8 * P + ns * 8 + 28 * P + 24 * P
    if kernel == "k_link":
        return U * 28
    if kernel == "k_pairs":
        # per pair: own id, partner, history read, force and torque of the lower
        # sphere; per sphere pair the partner's torque; per contact the history
        # write; compulsory per-sphere and per-clump gathers (owner, template
        # sphere, material; the clump record)
        return P * (8 + 24 + v + t) + U * t + C * 24 + ns * (8 + mat) + nc * 128
    if kernel == "k_reduce_waves":
        # per upper entry: link, the pair's force and the partner's torque; per
        # pair: force and torque of the lower sphere; per sphere: clump position
        # and segment bounds (+ margin for the guard on a detection's step:
        # later steps test a per-clump bound first); per clump: record read and
        # write, template, scene, prescribed-motion index (+ its pose at the last
        # detection for the guard, + acceleration envelope when learned)
        return (U * (4 + v + t) + P * (v + t) + ns * (20 + (4 * det_frac if guard else 0)) +
                nc * (268 + (64 if guard else 0) + (4 if learned else 0)))
    if kernel in ("k_scan_reduce", "k_scan_final"):
        return cells * (4 if kernel == "k_scan_reduce" else 8)
    if kernel == "k_detect_begin":
        return cells * 8
    return 0.0


# Per-sphere-step bytes of the method itself, term by term as the hot-path
# scope table's measurement section states them (a1 pose, a2 binning, a3
# narrow phase, a5 history remap, a7 force, a8 reduction, a9 integration),
# with p true contact pairs and p_m candidate pairs per sphere.
def survey_step_bytes(p: float, p_m: float, k: float, deferred: bool) -> float:
    """B_plain = 454 + 220 p (detection every step, no margin);
    B_del = 234 + 148 p + 8 (p_m - p) + (244 + 72 p_m) / k."""
    if not deferred:
        return 454.0 + 220.0 * p
    return 234.0 + 148.0 * p + 8.0 * (p_m - p) + (244.0 + 72.0 * p_m) / k


def survey_kernel_bytes(kernel: str, st: dict) -> float:
    """The same terms per launch of the kernel that carries them: k_reduce_waves
    a8 + a9 (+ the guard's 24 B per sphere when detection is deferred), k_pairs
    a7, k_narrow a3 and k_carry a5 (per detection).  0 for a kernel the terms
    do not name."""
    ns = st["spheres"]
    p = st["contact_sides"] / 2.0 / ns
    p_m = st["pairs"] / ns
    if kernel == "k_reduce_waves":
        return ns * ((16 + 56 * p) + 84 + (24 if st["guard"] else 0))
    if kernel == "k_pairs":
        return ns * (60 + 92 * p + 8 * (p_m - p))
    if kernel == "k_narrow":
        return ns * (64 + 8 * p_m)
    if kernel == "k_carry":
        return ns * 64 * p_m
    return 0.0


def make_scene(desc, mode, mlp=None, detect=None, precision="fp32"):
    """The scene as the benchmark times it: FP32 force arithmetic (unless
    `precision` says otherwise), detection `mode`."""
    from paper_2307_03445_amd._lib import Scene
    sc = Scene(desc, precision=precision)
    if mode == "learned":
        sc.set_mlp(mlp)
    if mode != "plain":
        sc.set_detection(mode, **(detect or DETECT))
    return sc


class WheelCosim:
    """The multibody side of a co-simulation with a wheel mesh (Sec. 5.2): a
    rigid wheel with a free vertical degree of freedom under a total load,
    driven at fixed forward and angular velocities.  Every `every` steps it
    records one step's boundary contacts, reads the force the spheres exert
    on the wheel, and prescribes the wheel's vertical velocity for the next
    interval (explicit Euler over the interval).  Works on a GPU scene or on
    the oracle (same exchanges, same numbers)."""

    def __init__(self, mesh=0, mass=10.0, load=100.0, every=10, h=1e-6):
        self.mesh, self.mass, self.load, self.every, self.h = mesh, mass, load, every, h
        self.since = 0
        self.exchanges = 0
        self.exchange_s = 0.0
        self.last_force = None

    def advance(self, sim, n, step=None):
        step = step or (lambda k: sim.step(k))
        gpu = hasattr(sim, "record_next_step")
        done = 0
        while done < n:
            k = min(self.every - 1 - self.since, n - done)
            if k > 0:
                step(k)
                done += k
                self.since += k
                continue
            if gpu:
                sim.record_next_step(walls_only=True)
                step(1)
                t0 = time.perf_counter()
                F, _ = sim.mesh_forces()
            else:
                sim.eval()
                F, _ = sim.mesh_forces()
                sim.step(1)
                t0 = time.perf_counter()
            done += 1
            st = sim.mesh_state()[self.mesh].copy()
            st[9] = st[9] + (self.every * self.h) * ((F[self.mesh][2] - self.load) / self.mass)
            sim.set_mesh_state(self.mesh, st)
            self.exchange_s += time.perf_counter() - t0
            self.last_force = F[self.mesh].copy()
            self.since = 0
            self.exchanges += 1


def _steps_reporting_misses(sc, n, label):
    """Advance n steps; an audit that finds a missed contact still ran its
    steps: report it instead of stopping the benchmark."""
    from paper_2307_03445_amd._lib import CdemError
    try:
        sc.step(n)
    except CdemError as e:
        if e.code != -5:
            raise
        log(f"[{label}] audit reported missed contacts: {e}")


def run_path(desc, mode, steps, warmup, mlp=None, graph=0, label=None, detect=None, precision="fp32",
             overlap=False, cosim=None):
    """Time `steps` steps of one path after warmup and the autotuner.

    Inside the timed region only the roofline kernel is bracketed by events
    (events around every kernel cost about 5 % of a step); a path replayed
    from a captured graph carries no events at all.  After the window, two
    untimed passes of one audit period each: the first times only the
    periodic audit's chain (its binning, exact check and fold, bracketed as
    one), the second every kernel for the per-kernel table."""
    import torch
    label = label or mode
    detect = detect or DETECT
    period = detect["audit_period"] if mode != "plain" else 0
    sc = make_scene(desc, mode, mlp, detect, precision)
    if cosim:  # every step of the warmup and of the window goes through the exchanges
        advance = lambda n: cosim.advance(sc, n, step=lambda k: _steps_reporting_misses(sc, k, label))
    else:
        advance = lambda n: _steps_reporting_misses(sc, n, label)
    t0 = time.perf_counter()
    advance(warmup)
    # bin size and launch shape from the library's autotuner (its trials are
    # ordinary steps, each of one detection and the steps up to the next at
    # the interval bound), then steps to settle before timing
    tune = sc.autotune(detect["k_max"] if mode != "plain" else 5)
    if overlap:  # the next active set built on a second stream while the steps go on
        sc.set_detection(mode, **dict(detect, overlap=True))
    if graph:
        sc.set_graph(graph)
    advance(warmup)
    log(f"[{label}] warmup {2 * warmup} steps and autotuning ({tune}): {time.perf_counter() - t0:.2f} s")
    c0 = sc.counts()
    if not graph:
        sc.profile(True, only=(ROOFLINE_KERNEL,))
    ex0 = (cosim.exchanges, cosim.exchange_s) if cosim else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(period, steps - done) if period else steps - done
        advance(n)
        done += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cos = None
    if cosim:
        cos = dict(every=cosim.every, exchanges=cosim.exchanges - ex0[0],
                   exchange_ms=(cosim.exchange_s - ex0[1]) * 1e3, wheel_force=cosim.last_force.tolist())
    prof_timed = sc.profile_read() if not graph else {}
    c1 = sc.counts()
    contact_sides = sc.last_step_contacts()
    window = {k: c1[k] - c0[k] for k in ("steps", "detections", "guard_trips", "fallbacks", "audits", "missed")}
    if graph:
        sc.set_graph(0)
    audit = None
    if period:
        # one audit period, only the audit chain timed: the cost of one audit
        # (its kernels also launch, empty, on the other steps of the period)
        a0 = sc.counts()
        sc.profile(True, only=("audit_total",))
        _steps_reporting_misses(sc, period, label)
        pa = sc.profile_read()
        a1 = sc.counts()
        n_a, ms_a = pa.get("audit_total", (0, 0.0))
        audit = dict(steps=period, audits=a1["audits"] - a0["audits"], missed=a1["missed"] - a0["missed"],
                     true_contacts_seen=a1["audit_contacts"], chain_ms=ms_a, chain_launches=n_a)
    # every kernel, over one audit period more (or 20 steps of the plain path)
    sc.profile(True)
    _steps_reporting_misses(sc, period or min(20, steps), label)
    prof = sc.profile_read()
    sc.profile(False)
    c2 = sc.counts()
    sc.close()
    dets = window["detections"]
    log(f"[{label}] {steps} steps in {dt:.3f} s; window {window}; candidates {c1['candidates']}; "
        f"contact sides {contact_sides}; audit {audit}")
    for k, (n, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"    {k:22s} launches {n:6d} total {ms:9.2f} ms  avg {ms / n * 1e3:9.1f} us")
    return dict(seconds=dt, prof=prof, prof_timed=prof_timed, counts=c1, detections=dets, window=window,
                contact_sides=contact_sides, guard_trips=window["guard_trips"], tune=tune, steps=steps,
                audit=audit, pass_detections=c2["detections"] - c1["detections"], graph=graph, cosim=cos)


KERNEL_SOURCES = ("paper_2307_03445_amd/csrc/kernels.hip", "paper_2307_03445_amd/csrc/cdem_internal.h",
                  "paper_2307_03445_amd/csrc/mlp_dev.h", "paper_2307_03445_amd/csrc/step_dev.h",
                  "paper_2307_03445_amd/csrc/pair_dev.h")
COUNTERS = os.path.join(ROOT, "profiles", "counters_rover_bed.json")


def kernel_source_hash() -> str:
    """Fingerprint of the kernel sources with comments and layout removed
    (a change of wording leaves the compiled kernels, and so the counters
    taken on them, as they were)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
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


def path_stats(res, desc_stats, mode):
    cnt = res["counts"]
    return dict(desc_stats, pairs=cnt["pairs"], upper=cnt["candidates"] - cnt["pairs"],
                contact_sides=res["contact_sides"], guard=(mode != "plain"), learned=(mode == "learned"),
                detect_fraction=min(1.0, res["detections"] / max(1, res["steps"])))


def roofline(res, desc_stats, mode, counters=True):
    """Roofline entry of the dominant kernel: `achieved` from the per-unit
    bytes of the hot-path scope table's measurement section (per sphere,
    with the measured contacts and candidates per sphere) times the spheres
    a launch processes, divided by the kernel's mean launch duration (HIP
    events inside the timed region when it is the kernel timed there);
    `achieved_layout` the same with this library's own record layout.
    `traffic` only for the workload the committed counters were taken on
    (`counters`; null for the other workloads)."""
    prof = res["prof"]
    k, (n, ms) = max(prof.items(), key=lambda kv: kv[1][1] if kv[0] != "audit_total" else -1)
    timed = k in res["prof_timed"]
    if timed:
        n, ms = res["prof_timed"][k]
    st = path_stats(res, desc_stats, mode)
    # a detection kernel early-exits when no detection is due: count only real launches
    launches = n
    if k == "k_pose":  # works on the steps that detect or audit
        launches = max(1, res["pass_detections"] + (res["audit"] or {}).get("audits", 0))
    if k in ("k_narrow", "k_narrow_fb", "k_narrow_base", "k_narrow_rows", "k_link", "k_carry", "k_cell_count",
             "k_cell_scatter",
             "k_detect_begin", "k_scan_reduce", "k_scan_final"):
        launches = max(1, res["detections"] if timed else res["pass_detections"])
    avg_s = ms / 1e3 / launches
    b = survey_kernel_bytes(k, st)
    bl = layout_bytes(k, st)
    gbs = b / avg_s / 1e9 if b else None
    gbl = bl / avg_s / 1e9 if bl else None
    return dict(bound="hbm", kernel=k, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(gbs / HBM_PEAK_GBS) if gbs else None, traffic=measured_traffic(k) if counters else None,
                bytes_per_launch=b, avg_launch_us=avg_s * 1e6, timed_region=timed,
                achieved_layout=gbl, frac_layout=(gbl / HBM_PEAK_GBS) if gbl else None,
                bytes_per_launch_layout=bl)


def path_line(res, ns, stats, mode):
    """One path's numbers: the window's rate with and without the periodic
    audit's cost amortised over its period, the window's counters, and the
    whole step's bytes by the scope table's per-unit model against the HBM
    peak."""
    dt, steps = res["seconds"], res["steps"]
    sps_no_audit = ns * steps / dt
    audit_ms_per_step = 0.0
    if res["audit"] and res["audit"]["audits"] > 0:
        # the chain's time over the period (one audit, empty launches on the
        # other steps, which the window already pays: counted twice here)
        audit_ms_per_step = res["audit"]["chain_ms"] / res["audit"]["steps"]
    sps = ns * steps / (dt + steps * audit_ms_per_step / 1e3)
    st = path_stats(res, stats, mode)
    p = st["contact_sides"] / 2.0 / ns
    p_m = st["pairs"] / ns
    k_eff = steps / max(1, res["window"]["detections"])
    B = survey_step_bytes(p, p_m, k_eff, mode != "plain")
    return {"sphere_steps_per_s": sps, "sphere_steps_per_s_no_audit": sps_no_audit,
            "ms_per_step": dt / steps * 1e3, "audit_ms_per_step": audit_ms_per_step,
            "audit": res["audit"], "window": res["window"], "candidates": res["counts"]["candidates"],
            "pairs": res["counts"]["pairs"], "contact_sides": res["contact_sides"],
            "missed_total": res["counts"]["missed"], "autotune": res["tune"], "graph_steps": res["graph"],
            "p": p, "p_m": p_m, "k_effective": k_eff, "step_bytes_per_sphere": B,
            "step_frac_of_hbm_peak": B * sps / (HBM_PEAK_GBS * 1e9)}


def cpu_baseline(seconds_target=12.0, cores=None):
    import oracle
    from paper_2307_03445_amd import inputs as I
    oracle.build(force=False)
    if cores is None:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(cores)
    d = I.walled_box()
    o = oracle.Oracle(d)
    o.step(5)
    t0 = time.perf_counter()
    o.step(10)
    per = (time.perf_counter() - t0) / 10
    n = int(max(10, min(20000, seconds_target / max(per, 1e-6))))
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--clumps", type=int, default=11_000_000)
    ap.add_argument("--modes", default="plain,fixed,learned,learned_overlap,learned_graph,learned_fixed_point,"
                                       "mesh_cosim,batched,precision",
                    help="paths to time: plain, fixed, learned (rover bed), learned_overlap (the learned path "
                         "with the next active set built on a second stream while the steps go on), "
                         "learned_graph (the learned path replayed from captured graphs), learned_fixed_point "
                         "(the learned path with fixed-point clump positions, 2^-40 m), mesh_cosim (the bed with "
                         "the wheel as a triangle mesh, co-simulated: one exchange of wheel force and velocity "
                         "every 10 steps), batched (256 funnel scenes, learned, graphs), precision (the "
                         "4M-clump drum, learned, all-FP64 vs FP32 force arithmetic)")
    ap.add_argument("--mlp", default=None, help="npz with envelope-MLP parameters (default: the package's "
                                                "trained weights, else train now)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--funnel-settle-s", type=float, default=0.05,
                    help="simulated seconds the funnel batch runs (at h = 5e-6 s) before it is timed")
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
    modes = args.modes.split(",")
    rover_modes = [m for m in modes if m in ("plain", "fixed", "learned", "learned_overlap", "learned_graph",
                                             "learned_fixed_point")]
    mlp, mlp_info = None, None
    if any(m in modes for m in ("learned", "learned_graph", "learned_fixed_point", "mesh_cosim", "batched",
                                "precision")):
        from paper_2307_03445_amd import train
        path = args.mlp or train.WEIGHTS
        if os.path.exists(path):
            mlp = np.load(path)["params"].astype(np.float32)
            mlp_info = f"loaded {os.path.relpath(path, ROOT)}"
    results, desc = {}, None
    px = pq = None
    if rover_modes or "precision" in modes or "mesh_cosim" in modes:
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
        if mlp is None and (any(m.startswith("learned") for m in rover_modes) or "mesh_cosim" in modes):
            from paper_2307_03445_amd import train
            t1 = time.perf_counter()
            mlp, info = train.train(px, pq, log=log)
            mlp_info = f"trained now in {time.perf_counter() - t1:.1f} s: {info}"
    if rover_modes:
        desc = I.rover_bed(px, pq, n_clumps=args.clumps)
        log(f"workload: {desc.n_clumps} clumps, {desc.n_spheres} spheres, built in {time.perf_counter() - t0:.1f} s")
        log(f"envelope MLP: {mlp_info}")
        for mode in rover_modes:
            base = "learned" if mode.startswith("learned") else mode
            d = dataclasses.replace(desc, pos_exp=40) if mode == "learned_fixed_point" else desc
            results[mode] = run_path(d, base, args.steps, args.warmup, mlp=mlp,
                                     graph=args.steps if mode == "learned_graph" else 0, label=mode,
                                     overlap=mode == "learned_overlap")
    mesh_cosim = None
    if "mesh_cosim" in modes:
        t0 = time.perf_counter()
        mdesc = I.rover_bed(px, pq, n_clumps=args.clumps, wheel="mesh")
        log(f"mesh co-simulation workload: {mdesc.n_clumps} clumps, {mdesc.n_spheres} spheres, wheel of "
            f"{mdesc.n_tri} triangles, built in {time.perf_counter() - t0:.1f} s")
        rm = run_path(mdesc, "learned", args.steps, args.warmup, mlp=mlp, label="mesh_cosim",
                      cosim=WheelCosim(mesh=0, mass=10.0, load=100.0, every=10, h=mdesc.h))
        mstats = dict(spheres=mdesc.n_spheres, clumps=mdesc.n_clumps, fp32=True, bins=rm["counts"]["bins"])
        mesh_cosim = dict(path_line(rm, mdesc.n_spheres, mstats, "learned"),
                          workload=f"rover-scale bed of {mdesc.n_clumps} clumps, {mdesc.n_spheres} spheres, with the "
                                   f"wheel as a mesh of {mdesc.n_tri} triangles (R = 0.254 m rim, 12 grousers) "
                                   f"driven at slip 0.2 and co-simulated: every 10 steps one step's boundary "
                                   f"contacts are recorded, the wheel force read and its vertical velocity "
                                   f"prescribed (10 kg, 100 N load), learned interval",
                          cosim=rm["cosim"], roofline=roofline(rm, mstats, "learned", counters=False))
    batched = None
    if "batched" in modes:
        t0 = time.perf_counter()
        bdesc = I.funnel_batch()
        # the scenes mid-discharge: off the spawn lattice, packed into the
        # funnels and flowing through the outlets
        bdesc, binfo = prep.settle_funnels(bdesc, seconds=args.funnel_settle_s)
        log(f"batched workload: {bdesc.n_scenes} funnel scenes, {bdesc.n_clumps} clumps, {bdesc.n_spheres} "
            f"spheres, built and run {args.funnel_settle_s} s into the discharge in {time.perf_counter() - t0:.1f} s "
            f"({binfo})")
        rb = run_path(bdesc, "learned", args.steps, args.warmup, mlp=mlp, graph=args.steps, label="batched")
        bstats = dict(spheres=bdesc.n_spheres, clumps=bdesc.n_clumps, fp32=True, bins=rb["counts"]["bins"])
        batched = dict(path_line(rb, bdesc.n_spheres, bstats, "learned"),
                       workload=f"{bdesc.n_scenes} independent funnel scenes of 2k-60k clumps (log-uniform), "
                                f"{bdesc.n_clumps} clumps, {bdesc.n_spheres} spheres, {args.funnel_settle_s} s "
                                f"into the discharge, learned interval, one captured graph of {args.steps} steps "
                                f"per replay",
                       roofline=roofline(rb, bstats, "learned", counters=False))
    precision = None
    if "precision" in modes:
        t0 = time.perf_counter()
        ddesc = I.drum_bed(px, pq)
        log(f"precision workload: drum of {ddesc.n_clumps} clumps, {ddesc.n_spheres} spheres, built in "
            f"{time.perf_counter() - t0:.1f} s")
        precision = {"workload": f"rotating drum (R = 0.4 m, L = 3 m, 2 rad/s) filled with {ddesc.n_clumps} clumps, "
                                 f"{ddesc.n_spheres} spheres (copies of the settled bed patch), learned interval"}
        for prec in ("fp64", "fp32"):
            rp = run_path(ddesc, "learned", args.steps, args.warmup, mlp=mlp, label=f"drum-{prec}",
                          precision=prec)
            pstats = dict(spheres=ddesc.n_spheres, clumps=ddesc.n_clumps, fp32=(prec == "fp32"),
                          bins=rp["counts"]["bins"])
            precision[prec] = dict(path_line(rp, ddesc.n_spheres, pstats, "learned"),
                                   roofline=roofline(rp, pstats, "learned", counters=False))
        precision["fp32_over_fp64"] = (precision["fp32"]["sphere_steps_per_s"] /
                                       precision["fp64"]["sphere_steps_per_s"])
    if not results:
        line = {"metric": METRIC, "batched": batched, "precision": precision, "mesh_cosim": mesh_cosim}
        print(json.dumps(line), flush=True)
        return
    main_mode = "learned" if "learned" in results else (
        "fixed" if "fixed" in results else next(iter(results)))
    r = results[main_mode]
    stats = dict(spheres=desc.n_spheres, clumps=desc.n_clumps, fp32=True, bins=r["counts"]["bins"])
    paths = {m: path_line(v, desc.n_spheres, stats, "plain" if m == "plain" else "learned" if m.startswith(
        "learned") else m) for m, v in results.items()}
    main = paths[main_mode]
    line = {
        "metric": METRIC,
        "value": main["sphere_steps_per_s"],
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
                               f"at slip 0.2, h=1e-6 s", "detection": main_mode,
                   "value_includes": "the periodic audit (every 100 steps) amortised over its period"},
        "value_no_audit": main["sphere_steps_per_s_no_audit"],
        "paths": paths,
        "envelope_mlp": mlp_info,
        "roofline": roofline(r, stats, "plain" if main_mode == "plain" else "learned"),
    }
    if "plain" in results and main_mode != "plain":
        line["speedup_vs_plain"] = main["sphere_steps_per_s"] / paths["plain"]["sphere_steps_per_s"]
    if batched:
        line["batched"] = batched
    if mesh_cosim:
        line["mesh_cosim"] = mesh_cosim
    if precision:
        line["precision"] = precision
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
        line["cpu_baseline_1core"] = cpu_baseline(seconds_target=10.0, cores=1)
        line["gpu_on_cpu_sample"] = gpu_on_cpu_sample()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
