"""Benchmark of the explicit bioheat stepper on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2|3|4|5|6|7]

A bench step is one rfa_step call that advances the workload by its full
simulated duration (all per-step work: conduction, perfusion, RF source,
held voxels, float-float Euler update, Arrhenius damage and latch,
per-step diagnostics), with the grid's inputs resident in HBM.  The default
workload is the single-instance heterogeneous case: 128^3 voxels at 0.5 mm,
liver with a tumour and 3-6 vessels, straight needle, 1000 steps of
0.01 s.  --config 3 runs the 256^3 umbrella-needle case (6000 steps);
--config 4 the batched sweep, --config 5 the differentiation workload
(forward + adjoint), --config 6 the breathing-motion view of a 256^3
temperature image (one warp per step) and --config 7 one GPU's share of
the 256^3 case (its middle y slab, 256x34x256).

Prints one JSON line: voxel-updates/s over the timed steps, the step
kernel's roofline (algorithmic bytes per launch over its HIP-event-timed
average duration), and the FP64 oracle timed on this host's cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GVoxel-updates/s + % HBM roofline (fwd, fwd+adjoint) vs plain stepper, "
          "ΔT≤1e-4K")
# Minimum bytes one voxel-step must move through HBM (per step, one pass):
# float-float state read + write (8 + 8), class byte (1), source increment
# (4), damage integral read + write (4 + 4).
BYTES_PER_VOXEL_STEP = 29
# Adjoint step with a perfusion field: lambda read + write (4 + 4), theta^n
# (4), class (1), weight (4), perfusion factor (4), the two accumulators
# read + write (8 + 8).
ADJ_BYTES_PER_VOXEL_STEP = 37
# Adjoint launch on the 128^3 differentiation grid: 8-row tiles of 64 z, 16 x
# planes per work-group, 256 work-groups.
ADJ_PLAN = {"rows": 8, "z": 64, "x_planes": 16, "workgroups": 256}
HBM_PEAK_GBPS = 8000.0
# Step-kernel launches per HIP-event-timed block (one event pair per block).
# A divisor of the library's 64-step diagnostic reduction period keeps those
# reductions between blocks; 64 rather than 16 keeps the event records'
# own cost (about 3 % of a 13 us launch) out of the measured throughput.
TIME_PERIOD = 64
# Sources that define each step kernel's device code; a committed traffic
# record applies while they hash as they did when its counters were taken.
_CSRC = "paper_1907_05709_amd/csrc/"
_SHARED = ("rfa_tile_common.h", "rfa_device.h", "rfa_kernels.h")
KERNEL_SOURCES = {
    "k_step_wide": ("rfa_wide.hip",) + _SHARED,
    "k_step_tiled": ("rfa_tiled.hip", "rfa_tiled.h") + _SHARED,
    "k_step_batch": ("rfa_tiled.hip", "rfa_tiled.h") + _SHARED,
    "k_warp": ("rfa_warp.hip", "rfa_warp.h") + _SHARED,
    "k_adjoint_tiled": ("rfa_adjoint.hip", "rfa_adjoint.h", "rfa_tiled.h") + _SHARED,
}


def kernel_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, _CSRC + f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# One-step launch plans (z voxels per lane, tile rows, x planes per
# work-group) of the single-grid workloads: the fastest of rfa_tune's
# candidates on the MI355X, fixed so that the committed counter summaries
# refer to the timed launch shape.
PLANS = {2: (2, 8, 4), 3: (4, 4, 32), 7: (2, 4, 4)}


def kernel_name(plan: dict) -> str:
    if plan["kernel"] != 2:
        return "k_step_naive"
    if plan["depth"] == 2:
        return "k_step_tiled2"
    return "k_step_wide" if plan["z_vec"] > 1 else "k_step_tiled"


def workload(config: int):
    from paper_1907_05709_amd import workloads as W
    if config == 2:
        case = W.case_straight()
        name = ("straight-needle liver/tumour/vessels 128^3 @0.5mm, 1000 x 0.01 s, "
                "P~U(15,40) W (seed 2000)")
    elif config == 3:
        case = W.case_umbrella()
        name = ("9-tine umbrella liver/tumour/vessels 256^3 @0.5mm, 6000 x 0.01 s, "
                "60 W (seed 3000)")
    elif config == 7:
        # the middle y slab [111, 145) of the 256^3 umbrella case: one GPU's
        # share of eight (32 rows) plus the two halo rows, held here; voxel
        # centres coincide with the full grid's, the needle's power is
        # normalised over the slab.  Slabs across y keep the full x extent
        # for the kernels' x-march (thin x slabs cut it short).
        import dataclasses
        import numpy as np
        full = W.case_umbrella()
        case = dataclasses.replace(full, shape=(256, 34, 256),
                                   labels=np.ascontiguousarray(full.labels[:, 111:145]))
        name = ("y slab 256x34x256 of the 256^3 umbrella case (one GPU's share of 8: 32 rows "
                "+ 2 halo rows), 6000 x 0.01 s")
    else:
        raise SystemExit("--config must be 2, 3, 4, 5, 6 or 7")
    return case, name


def traffic_record(config: int, plan: dict, kernel: str, name: str = ""):
    """Bytes per launch below L2 from committed rocprofv3 counter summaries,
    if they were taken on the kernel's current sources and launch plan."""
    path = os.path.join(ROOT, "profiles", name or f"traffic_step_config{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (kernel not in KERNEL_SOURCES or rec.get("kernel_hash") != kernel_hash(kernel)
            or rec.get("plan") != plan):
        return None
    return rec.get("hbm_bytes_per_launch")


def with_traffic_rate(roofline: dict) -> dict:
    """Add the measured memory-side rate: the committed below-L2 bytes per
    launch over the live average launch duration, and its fraction of the
    peak (null without a valid traffic record)."""
    t, us = roofline.get("traffic"), roofline.get("avg_launch_us")
    rate = t / (us * 1e-6) / 1e9 if t and us else None
    roofline["traffic_GBps"] = round(rate, 1) if rate else None
    roofline["traffic_frac"] = round(rate / roofline["peak"], 4) if rate else None
    return roofline


def cpu_baseline(case, sample_steps: int):
    """The FP64 oracle (as is) on the host cores: sample_steps steps of the
    same workload, with its per-step diagnostics."""
    from oracle import oracle as O
    O.build(force=False)
    q = O.source(case)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    O.run(case, n_steps=sample_steps, q=q, diag=True)
    dt = time.perf_counter() - t0
    gvox = case.n_voxels * sample_steps / dt / 1e9
    return {"value": gvox, "unit": "GVoxel-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample_steps} of {case.n_steps} steps of the same workload "
                      f"({'x'.join(str(n) for n in case.shape)}), FP64 with per-step diagnostics, "
                      f"{dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle sample steps (0 = size for ~15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="re-tune the launch plan instead of the fixed one")
    ap.add_argument("--plan", default="",
                    help="launch plan zv,ty,xc for --config 2/3 instead of the fixed one")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="override the workload's time steps per bench step (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1907_05709_amd import rfa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_adjoint(args)
    if args.config == 6:
        return bench_warp(args)
    case, name = workload(args.config)
    if args.time_steps > 0:
        case.n_steps = args.time_steps
        name += f" [profiling run: {args.time_steps} time steps per bench step]"
    # one step per launch: the HBM-bound kernel whose roofline is reported
    zv, ty, xc = (tuple(int(t) for t in args.plan.split(",")) if args.plan
                  else PLANS[args.config])
    g = rfa.Grid(case.shape, case.spacing, device=False, depth=1, z_vec=zv, tile_y=ty,
                 tile_x=xc, time_kernels=TIME_PERIOD)
    g.load_case(case)
    if args.tune:
        g.tune(case.dt, reps=10)
    plan = g.plan()
    for _ in range(args.warmup):
        g.step(case.n_steps, case.dt, diag=True)
    g.kernel_stats()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diag = None
    for _ in range(args.steps):
        diag = g.step(case.n_steps, case.dt, diag=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches, vsteps = g.kernel_stats()
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    g.close()

    vox_updates = case.n_voxels * case.n_steps * args.steps
    value = vox_updates / wall / 1e9
    avg_ms = kms / launches
    bytes_per_launch = BYTES_PER_VOXEL_STEP * case.n_voxels
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = traffic_record(args.config, plan, kernel_name(plan))
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "grid": list(case.shape), "time_steps": case.n_steps,
                   "dt_s": case.dt, "state": "float-float f32 excess temperature",
                   "plan": plan},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "kernel": kernel_name(plan),
                     "avg_launch_us": round(avg_ms * 1e3, 3),
                     "launches_timed": launches, "bytes_per_launch": bytes_per_launch,
                     "copy_ceiling_GBps": round(copy_gbps, 1)},
        "diag_last_step": {k: diag[k] for k in ("t_max_C", "mono_violations", "residual_J")},
    }
    if not args.no_cpu:
        steps = args.cpu_steps
        if steps <= 0:
            steps = max(2, min(case.n_steps, int(2.0e9 / case.n_voxels)))
        out["cpu_baseline"] = cpu_baseline(case, steps)
    out["roofline"] = with_traffic_rate(out["roofline"])
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Planning sweep: 64 uneven grids (64^3..160^3, 0.5..1 mm, own needle,
    dt = 0.01 s (dx / 0.5 mm)^2), 2000 steps each; one bench step is one
    batched call advancing every grid by its 2000 steps (grids grouped to
    the last-level cache, each group's steps back to back, one hipGraph).
    The plain stepper (each grid stepped on its own, one after another) is
    timed beside it."""
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd import workloads as W

    n_steps = args.time_steps if args.time_steps > 0 else 2000
    cases = W.planning_sweep(64, n_steps=n_steps)
    grids = []
    for c in cases:
        g = rfa.Grid(c.shape, c.spacing)
        g.load_case(c)
        grids.append(g)
    total_vox = sum(c.n_voxels for c in cases)
    # plain stepper: every grid on its own, one after another
    for g, c in zip(grids, cases):
        g.step(min(n_steps, 20), c.dt, diag=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, c in zip(grids, cases):
        g.step(n_steps, c.dt, diag=False)
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    seq_value = total_vox * n_steps / seq_wall / 1e9

    b = rfa.Batch(grids, [c.dt for c in cases])
    if args.tune:
        b.tune(reps=20)
    for _ in range(args.warmup):
        b.step(n_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = 0.0
    for _ in range(args.steps):
        b.step(n_steps)
        ms, _ = b.last_time()
        dev_ms += ms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = total_vox * n_steps * args.steps / wall / 1e9
    plan = b.plan()
    # one launch per group and step (grids of a group share a launch; all of
    # the sweep's grids carry no perfusion field): device time of the graph
    # per launch, algorithmic bytes per launch averaged over the groups
    launches = plan["groups"] * n_steps * args.steps
    avg_launch_ms = dev_ms / launches
    bytes_per_launch = BYTES_PER_VOXEL_STEP * total_vox / plan["groups"]
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    b.close()
    for g in grids:
        g.close()
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"planning sweep: 64 grids 64^3..160^3 @0.5..1 mm, straight / "
                               f"3-tine / 9-tine needles, {n_steps} steps each, per-grid dt "
                               f"(seeds 4000..4063)",
                   "voxels": total_vox, "time_steps": n_steps, "batch_plan": plan,
                   "plain_stepper_GVox_s": round(seq_value, 3),
                   "batched_speedup_vs_plain": round(value / seq_value, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_record(4, plan, "k_step_batch"), "kernel": "k_step_batch",
                     "avg_launch_us": round(avg_launch_ms * 1e3, 3),
                     "bytes_per_launch": round(bytes_per_launch),
                     "note": "groups of grids sized to the 256 MB last-level cache run "
                             "their steps back to back; traffic counts bytes below L2, "
                             "which that cache may serve"},
    }
    out["roofline"] = with_traffic_rate(out["roofline"])
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Differentiation workload: 128^3 at 0.5 mm, 9-tine umbrella (60 W
    shared by length), 600 steps of 0.02 s, perfusion corrected by a 16^3
    B-spline lattice (all zero).  One bench step = reset, forward keeping the
    temperature of every step in HBM (5 GB), coverage loss and its gradient
    with respect to the damage integral (torch, on the GPU), adjoint to the 9
    tine powers and the 4096 lattice values.  value = simulated voxel-steps
    per second of forward + adjoint.  The checkpointed schedule (state every
    50 steps, each segment recomputed in the adjoint; same gradients, bitwise)
    is timed beside it."""
    import numpy as np
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd import workloads as W
    from paper_1907_05709_amd.autograd import coverage_loss

    n_steps = args.time_steps if args.time_steps > 0 else 600
    case = W.case_differentiation(n_steps=n_steps)
    m, ckpt = 16, 50
    g = rfa.Grid(case.shape, case.spacing, device=True, time_kernels=TIME_PERIOD)
    g.load_case(case)
    g.set_perfusion_bspline(np.zeros((m, m, m), np.float32))
    plan = g.plan()
    labels = torch.from_numpy(case.labels).cuda()
    vox = float(np.prod(case.spacing))

    def one_step(every=0):
        g.reset_state()
        g.forward_checkpointed(n_steps, case.dt, every)
        _, om, _ = g.damage()
        om.requires_grad_(True)
        loss = coverage_loss(om, labels, vox)
        (w,) = torch.autograd.grad(loss, om)
        dP, dc, _ = g.adjoint(w.float(), case.needle.n_tines, m)
        return float(loss.detach()), dP

    for _ in range(args.warmup):
        one_step()
    g.kernel_stats()
    g.adjoint_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, dP = one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches, _ = g.kernel_stats()
    adj_ms, adj_launches = g.adjoint_kernel_stats()
    # the checkpointed schedule, for comparison (not part of value)
    _, dP_ck = one_step(ckpt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        one_step(ckpt)
    torch.cuda.synchronize()
    ck_value = case.n_voxels * n_steps * args.steps / (time.perf_counter() - t1) / 1e9
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    g.close()
    value = case.n_voxels * n_steps * args.steps / wall / 1e9
    avg_ms = kms / max(launches, 1)
    # the perfusion factor field adds one float read per voxel-step
    bytes_per_launch = (BYTES_PER_VOXEL_STEP + 4) * case.n_voxels
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    adj_avg_ms = adj_ms / max(adj_launches, 1)
    adj_bytes = ADJ_BYTES_PER_VOXEL_STEP * case.n_voxels
    adj_achieved = adj_bytes / (adj_avg_ms * 1e-3) / 1e9
    fwd = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
           "kernel": kernel_name(plan) + " (forward)", "avg_launch_us": round(avg_ms * 1e3, 3),
           "launches_timed": launches, "bytes_per_launch": bytes_per_launch}
    adj = {"bound": "hbm", "achieved": round(adj_achieved, 1), "peak": HBM_PEAK_GBPS,
           "unit": "GB/s", "frac": round(adj_achieved / HBM_PEAK_GBPS, 4),
           "traffic": traffic_record(5, ADJ_PLAN, "k_adjoint_tiled",
                                     "traffic_adjoint_differentiation128.json"),
           "kernel": "k_adjoint_tiled (adjoint)", "avg_launch_us": round(adj_avg_ms * 1e3, 3),
           "launches_timed": adj_launches, "bytes_per_launch": adj_bytes,
           "copy_ceiling_GBps": round(copy_gbps, 1)}
    # the dominant kernel (more time in the timed region) carries the roofline
    dominant, other = (adj, fwd) if adj_ms > kms else (fwd, adj)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"differentiation: 9-tine umbrella 128^3 @0.5mm, {n_steps} x "
                               f"{case.dt} s, 16^3 B-spline perfusion lattice; value counts "
                               f"forward + adjoint per simulated step",
                   "trajectory": "every step's temperature kept in HBM, no recomputation",
                   "checkpointed_every_%d_GVox_s" % ckpt: round(ck_value, 3),
                   "checkpointed_gradients_equal": bool(np.array_equal(dP, dP_ck)),
                   "loss": loss, "dL_dP": [float(x) for x in dP]},
        "roofline": with_traffic_rate(dominant),
        "roofline_other_kernel": with_traffic_rate(other),
    }
    out["roofline"] = with_traffic_rate(out["roofline"])
    print(json.dumps(out), flush=True)


WARP_BYTES_PER_VOXEL = 20   # displacement (3 x 4) + source image (4) + output (4)
WARP_PLAN = {"threads": 256, "x_voxels_per_thread": 4}
WARP_FRAMES_PER_CYCLE = 100


def bench_warp(args):
    """Breathing-motion view (Eq. (eq:breathing)) of a 256^3 temperature
    image at 0.5 mm through a synthetic inverse-motion field of 12 mm
    cranio-caudal amplitude.  One bench step = one 4 s breathing cycle shown
    at 25 frames/s: 100 rfa_warp calls over the whole grid, the surrogate
    going 0 -> 1 -> 0, inputs and output resident in HBM.  value = output
    voxels per second."""
    import numpy as np
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd import workloads as W

    shape, spacing = (256, 256, 256), (0.5e-3,) * 3
    n = int(np.prod(shape))
    T = W.hot_field(shape, spacing)
    v_host = W.breathing_field(shape, spacing, amplitude_m=12e-3)
    g = rfa.Grid(shape, spacing, device=True)
    g.set_tissue(torch.ones(shape, dtype=torch.uint8, device="cuda"), W.standard_tissue())
    g.set_temperature(torch.from_numpy(T).cuda())
    v = torch.from_numpy(v_host).cuda()
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    betas = [W.breathing_surrogate(f / 25.0) for f in range(WARP_FRAMES_PER_CYCLE)]

    def cycle():
        for b in betas:
            g.warp(v, b, out=out)

    for _ in range(args.warmup):
        cycle()
    stream = torch.cuda.current_stream()    # the grid launches on this stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        cycle()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = args.steps * len(betas)
    avg_ms = e0.elapsed_time(e1) / launches
    # keyframe form, for comparison (not part of value): two phase fields
    # blended over the cycle, 32 algorithmic bytes per voxel
    v2 = torch.from_numpy(W.breathing_field(shape, spacing, amplitude_m=12e-3, seed=7001)).cuda()
    for b in betas[:10]:
        g.warp(v, 1.0 - b, out=out, v2=v2, beta2=b)
    e0.record(stream)
    for b in betas:
        g.warp(v, 1.0 - b, out=out, v2=v2, beta2=b)
    e1.record(stream)
    torch.cuda.synchronize()
    kf_ms = e0.elapsed_time(e1) / len(betas)
    del v2
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    g.close()
    value = n * launches / wall / 1e9
    bytes_per_launch = WARP_BYTES_PER_VOXEL * n
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    out_json = {
        "metric": "GVoxel/s of breathing-motion temperature views",
        "value": round(value, 3),
        "unit": "GVoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "breathing-motion warp: 256^3 @0.5mm temperature image (hot "
                               "spots to 900 degC), 12 mm synthetic inverse-motion field, "
                               "trilinear; one step = one 4 s breathing cycle, 100 frames",
                   "keyframe_two_fields": {"avg_launch_us": round(kf_ms * 1e3, 3),
                                           "GVox_s": round(n / (kf_ms * 1e-3) / 1e9, 1),
                                           "algorithmic_GBps": round(32 * n / (kf_ms * 1e-3) / 1e9, 1)}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_record(6, WARP_PLAN, "k_warp",
                                               "traffic_warp_breathing256.json"),
                     "kernel": "k_warp", "avg_launch_us": round(avg_ms * 1e3, 3),
                     "launches_timed": launches,
                     "bytes_per_launch": bytes_per_launch,
                     "copy_ceiling_GBps": round(copy_gbps, 1)},
    }
    if not args.no_cpu:
        from oracle.warp import warp as warp_oracle
        frames = max(1, args.cpu_steps or 8)
        t0 = time.perf_counter()
        for k in range(frames):
            warp_oracle(T, v_host, spacing, betas[(k * 37) % len(betas)])
        dt = time.perf_counter() - t0
        out_json["cpu_baseline"] = {
            "value": n * frames / dt / 1e9, "unit": "GVoxel/s", "cores": 1, "kind": "oracle",
            "sample": f"{frames} full 256^3 frames at spread phases of the cycle, FP64 "
                      f"numpy, {dt:.1f} s wall"}
    out_json["roofline"] = with_traffic_rate(out_json["roofline"])
    print(json.dumps(out_json), flush=True)


if __name__ == "__main__":
    main()
