"""Benchmark of the explicit bioheat stepper on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4|2|3|5|6|7]

The default workload (--config 4) is the batched planning sweep: 64 grids of
64^3..160^3 voxels at 0.5..1 mm, each with its own tissue, needle (straight,
3-tine or 9-tine umbrella), power and time step, 2000 steps each.  A bench
step is one rfa_batch_step call that advances every grid by its 2000 steps
(all per-step work: conduction, perfusion, RF source, held voxels,
float-float Euler update, Arrhenius damage and latch, per-step
diagnostics), with every input resident in HBM.  The plain stepper (each
grid stepped on its own, one after another) is timed beside it.  The
default line also carries two legs, each with its own roofline and CPU
baseline: the 256^3 umbrella-needle case (6000 steps, one grid) and the
differentiation workload (128^3, 600 steps, forward + adjoint with a
checkpoint every 50 steps).  --no-legs leaves them out.

Single workloads: --config 2 the 128^3 straight-needle case (1000 steps;
its state stays in the 256 MB last-level cache), 3 the 256^3 umbrella
case, 5 the differentiation workload, 6 the breathing-motion view of a
256^3 temperature image (one cycle of 100 warps per step) and 7 one GPU's
share of the 256^3 case (its middle y slab, 256x34x256).

Prints one JSON line: voxel-updates/s over the timed steps, the dominant
kernel's roofline (algorithmic bytes per launch over its HIP-event-timed
average duration), and the FP64 oracle timed on this host's cores (all of
them, and one) on a bounded sample of the same workload.
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
# float-float state read + write (8 + 8), class byte (1), damage integral
# read + write (4 + 4); plus the source increment (4) on the voxels where it
# is nonzero (the RF source's support: the kernels skip it elsewhere, where
# it is exactly 0).  29 B on a voxel of the support, 25 B off it.
BYTES_PER_VOXEL_STEP = 25
SOURCE_BYTES = 4
# Adjoint step with a perfusion field: lambda read + write (4 + 4), theta^n
# (4), class (1), weight (4), perfusion factor (4), the perfusion-gradient
# accumulator read + write (8); plus the source accumulator read + write (8)
# on the source's support only.
ADJ_BYTES_PER_VOXEL_STEP = 29
ADJ_SOURCE_BYTES = 8
# Adjoint launch on the 128^3 differentiation grid: 8-row tiles of 64 z, 16 x
# planes per work-group, 256 work-groups.
ADJ_PLAN = {"rows": 8, "z": 64, "x_planes": 16, "workgroups": 256}
# forward launch plan of the differentiation workload (z voxels per lane,
# tile rows, x planes): with a perfusion field the step kernel carries one
# more stream, and 4-row tiles of 8 planes run 12 % faster than the 8-row,
# 4-plane tiles the plain 128^3 step uses
ADJ_FWD_PLAN = (2, 4, 8)
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


# committed counter summaries, named for their kernel and workload
TRAFFIC_FILES = {2: "traffic_step_straight128.json", 3: "traffic_step_umbrella256.json",
                 4: "traffic_batch_sweep64.json", 5: "traffic_adjoint_differentiation128.json",
                 6: "traffic_warp_breathing256.json", 7: "traffic_step_yslab256.json"}


def traffic_record(config: int, plan: dict, kernel: str):
    """Bytes per launch below L2 from committed rocprofv3 counter summaries,
    if they were taken on the kernel's current sources and launch plan."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[config])
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


def _threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def cpu_baseline(cases, steps_all: int, steps_one: int, what: str):
    """The FP64 oracle (as is, with its per-step diagnostics) on the host
    cores: steps_all steps of every case in `cases` with all cores, then
    steps_one steps with one core.  The RF sources are computed first and
    not timed (setup)."""
    from oracle import oracle as O
    O.build(force=False)
    qs = [O.source(c) for c in cases]
    vox = sum(c.n_voxels for c in cases)
    threads = _threads()
    out = {}
    for n_thr, steps in ((threads, steps_all), (1, steps_one)):
        O.set_threads(n_thr)
        t0 = time.perf_counter()
        for c, q in zip(cases, qs):
            O.run(c, n_steps=steps, q=q, diag=True)
        dt = time.perf_counter() - t0
        out[n_thr == 1] = (vox * steps / dt / 1e9, dt)
    O.set_threads(threads)
    (v_all, t_all), (v_one, t_one) = out[False], out[True]
    return {"value": round(v_all, 4), "unit": "GVoxel-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what}: first {steps_all} steps with {threads} threads ({t_all:.1f} s "
                      f"wall), {steps_one} steps with 1 thread ({t_one:.1f} s); FP64 with "
                      f"per-step diagnostics; sources computed beforehand, untimed",
            "single_core": {"value": round(v_one, 5), "unit": "GVoxel-updates/s", "cores": 1}}


def roofline_dict(bytes_per_launch, avg_ms, kernel, **extra):
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": kernel,
         "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": round(bytes_per_launch)}
    r.update(extra)
    return r


def mix_ceiling(roof: dict, mix_gbps: float) -> dict:
    """The streaming rate of the step's byte mix without its stencil at the
    same size (rfa_mix_bandwidth), measured in the same run, and the
    kernel's achieved rate as a fraction of it."""
    return {"mix_ceiling_GBps": round(mix_gbps, 1),
            "frac_of_mix_ceiling": round(roof["achieved"] / mix_gbps, 4)}


def run_single(config: int, steps: int, warmup: int, plan_arg: str = "", tune: bool = False,
               time_steps: int = 0, cpu: bool = True, cpu_steps: int = 0) -> dict:
    """One grid stepped by its whole duration per bench step (configs 2, 3,
    7); returns the result fields of its JSON line."""
    import torch
    from paper_1907_05709_amd import rfa
    case, name = workload(config)
    if time_steps > 0:
        case.n_steps = time_steps
        name += f" [profiling run: {time_steps} time steps per bench step]"
    # one step per launch: the HBM-bound kernel whose roofline is reported
    zv, ty, xc = (tuple(int(t) for t in plan_arg.split(",")) if plan_arg else PLANS[config])
    g = rfa.Grid(case.shape, case.spacing, device=False, depth=1, z_vec=zv, tile_y=ty,
                 tile_x=xc, time_kernels=TIME_PERIOD)
    g.load_case(case)
    if tune:
        g.tune(case.dt, reps=10)
    plan = g.plan()
    for _ in range(warmup):
        g.step(case.n_steps, case.dt, diag=True)
    g.kernel_stats()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diag = None
    for _ in range(steps):
        diag = g.step(case.n_steps, case.dt, diag=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches, _ = g.kernel_stats()
    support = g.source_support()
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    mix_gbps = rfa.rfa_mix_bandwidth(case.n_voxels, 10)
    g.close()

    value = case.n_voxels * case.n_steps * steps / wall / 1e9
    avg_ms = kms / launches
    roof = roofline_dict(BYTES_PER_VOXEL_STEP * case.n_voxels + SOURCE_BYTES * support, avg_ms,
                         kernel_name(plan), launches_timed=launches,
                         copy_ceiling_GBps=round(copy_gbps, 1), source_support_voxels=support)
    roof.update(mix_ceiling(roof, mix_gbps))
    roof["traffic"] = traffic_record(config, plan, kernel_name(plan))
    # working set of one step: state in and out, class, source, damage
    ws_mb = case.n_voxels * (16 + 1 + 4 + 4) / 1e6
    if ws_mb < 200.0:
        roof["note"] = (f"the {ws_mb:.0f} MB working set stays in the 256 MB last-level "
                        f"cache: the launch is latency bound and 'hbm' names the peak it is "
                        f"priced against, not the level that serves it")
        roof["cache_resident"] = True
    out = {
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "ms_per_step": round(wall / steps * 1e3, 4),
        "config": {"workload": name, "grid": list(case.shape), "time_steps": case.n_steps,
                   "dt_s": case.dt, "state": "float-float f32 excess temperature",
                   "plan": plan},
        "roofline": with_traffic_rate(roof),
        "diag_last_step": {k: diag[k] for k in ("t_max_C", "mono_violations", "residual_J")},
    }
    if cpu:
        n = cpu_steps or max(2, min(case.n_steps, int(2.0e9 / case.n_voxels)))
        out["cpu_baseline"] = cpu_baseline([case], n, max(1, n // 25),
                                           f"the same workload ({'x'.join(map(str, case.shape))})")
    return out


def line(fields: dict, steps: int, warmup: int) -> dict:
    out = {"metric": METRIC, "value": fields["value"], "unit": fields["unit"], "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": fields["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    for k, v in fields.items():
        if k not in out:
            out[k] = v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle sample steps (0 = size for ~15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="--config 4: leave out the 256^3 and differentiation legs")
    ap.add_argument("--tune", action="store_true",
                    help="re-tune the launch plan instead of the fixed one")
    ap.add_argument("--plan", default="",
                    help="launch plan zv,ty,xc for --config 2/3 instead of the fixed one")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="override the workload's time steps per bench step (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(the build targets a single MI355X)"}))
        sys.exit(2)

    import torch
    from paper_1907_05709_amd import rfa  # noqa: F401  (fails loudly if not built)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == 4:
        out = line(bench_batch(args), args.steps, args.warmup)
        if not args.no_legs:
            out["legs"] = {
                "umbrella256": run_single(3, steps=2, warmup=1, cpu=not args.no_cpu,
                                          cpu_steps=60),
                "differentiation128": bench_adjoint(args, steps=3, warmup=1),
            }
        print(json.dumps(out), flush=True)
        return
    if args.config == 5:
        print(json.dumps(line(bench_adjoint(args, args.steps, args.warmup), args.steps,
                              args.warmup)), flush=True)
        return
    if args.config == 6:
        return bench_warp(args)
    if args.config not in (2, 3, 7):
        raise SystemExit("--config must be 2, 3, 4, 5, 6 or 7")
    fields = run_single(args.config, args.steps, args.warmup, args.plan, args.tune,
                        args.time_steps, cpu=not args.no_cpu, cpu_steps=args.cpu_steps)
    print(json.dumps(line(fields, args.steps, args.warmup)), flush=True)


# Planning-sweep instances timed by the oracle for the CPU baseline (one in
# eight, all three needle types and the size range) and their steps.
SWEEP_CPU_SAMPLE = tuple(range(0, 64, 8))


def bench_batch(args) -> dict:
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
    # plain stepper: every grid on its own, one after another; both legs
    # compute the per-step diagnostics, as every other bench step does
    for g, c in zip(grids, cases):
        g.step(min(n_steps, 20), c.dt, diag=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, c in zip(grids, cases):
        g.step(n_steps, c.dt, diag=True)
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    seq_value = total_vox * n_steps / seq_wall / 1e9

    b = rfa.Batch(grids, [c.dt for c in cases])
    if args.tune:
        b.tune(reps=20)
    for _ in range(args.warmup):
        b.step(n_steps, diag=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = 0.0
    for _ in range(args.steps):
        diag = b.step(n_steps, diag=True)
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
    support = sum(g.source_support() for g in grids)
    bytes_per_launch = (BYTES_PER_VOXEL_STEP * total_vox + SOURCE_BYTES * support) / plan["groups"]
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    b.close()
    for g in grids:
        g.close()
    mix_gbps = rfa.rfa_mix_bandwidth(total_vox // plan["groups"], 10)
    roof = roofline_dict(bytes_per_launch, avg_launch_ms, "k_step_batch",
                         launches_timed=launches, copy_ceiling_GBps=round(copy_gbps, 1),
                         source_support_voxels=support,
                         note="groups of grids sized to the 256 MB last-level cache run "
                              "their steps back to back; traffic counts bytes below L2, "
                              "which that cache may serve; the mix ceiling is taken over "
                              "one average group's voxels")
    roof.update(mix_ceiling(roof, mix_gbps))
    roof["traffic"] = traffic_record(4, plan, "k_step_batch")
    out = {
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "config": {"workload": f"planning sweep: 64 grids 64^3..160^3 @0.5..1 mm, straight / "
                               f"3-tine / 9-tine needles, {n_steps} steps each, per-grid dt "
                               f"(seeds 4000..4063)",
                   "voxels": total_vox, "time_steps": n_steps, "batch_plan": plan,
                   "state": "float-float f32 excess temperature",
                   "plain_stepper_GVox_s": round(seq_value, 3),
                   "batched_speedup_vs_plain": round(value / seq_value, 3)},
        "diag_last_call": {
            "t_max_C": round(max(d["t_max_C"] for d in diag), 3),
            "mono_violations": sum(d["mono_violations"] for d in diag),
            "worst_residual_of_budget": max(
                abs(d["residual_J"]) / (abs(d["injected_J"]) + abs(d["perfusion_J"])
                                        + abs(d["boundary_J"])) for d in diag)},
        "roofline": with_traffic_rate(roof),
    }
    if not args.no_cpu:
        sample = [cases[i] for i in SWEEP_CPU_SAMPLE]
        steps_all = args.cpu_steps or 100
        out["cpu_baseline"] = cpu_baseline(
            sample, steps_all, max(1, steps_all // 25),
            f"sweep instances {', '.join(map(str, SWEEP_CPU_SAMPLE))} "
            f"({sum(c.n_voxels for c in sample)} voxels) of the same sweep")
    return out


def bench_adjoint(args, steps: int, warmup: int) -> dict:
    """Differentiation workload: 128^3 at 0.5 mm, 9-tine umbrella (60 W
    shared by length), 600 steps of 0.02 s, perfusion corrected by a 16^3
    B-spline lattice (all zero).  One bench step = reset, forward with a
    checkpoint every 50 steps, coverage loss and its gradient with respect
    to the damage integral (torch, on the GPU), adjoint (each 50-step
    segment recomputed from its checkpoint) to the 9 tine powers and the
    4096 lattice values.  value = simulated voxel-steps per second of
    forward + adjoint.  The schedule that keeps every step's temperature in
    HBM (5 GB, no recomputation; same gradients, bitwise) is timed beside
    it, and its launches give the kernels' rooflines."""
    import numpy as np
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd import workloads as W
    from paper_1907_05709_amd.autograd import coverage_loss

    n_steps = args.time_steps if args.time_steps > 0 else 600
    case = W.case_differentiation(n_steps=n_steps)
    m, ckpt = 16, 50
    zv, ty, xc = ADJ_FWD_PLAN
    g = rfa.Grid(case.shape, case.spacing, device=True, time_kernels=TIME_PERIOD, z_vec=zv,
                 tile_y=ty, tile_x=xc)
    g.load_case(case)
    g.set_perfusion_bspline(np.zeros((m, m, m), np.float32))
    plan = g.plan()
    labels = torch.from_numpy(case.labels).cuda()
    vox = float(np.prod(case.spacing))

    def one_step(every):
        g.reset_state()
        g.forward_checkpointed(n_steps, case.dt, every)
        om = g.omega()
        om.requires_grad_(True)
        loss = coverage_loss(om, labels, vox)
        (w,) = torch.autograd.grad(loss, om)
        dP, dc, _ = g.adjoint(w.float(), case.needle.n_tines, m)
        return float(loss.detach()), dP

    def timed(every):
        for _ in range(warmup):
            one_step(every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            loss, dP = one_step(every)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, loss, dP

    wall, loss, dP = timed(ckpt)
    value = case.n_voxels * n_steps * steps / wall / 1e9
    # kept trajectory: value beside it, and the kernels' launch timing
    g.kernel_stats()
    g.adjoint_kernel_stats()
    kwall, _, dP_kept = timed(0)
    kept_value = case.n_voxels * n_steps * steps / kwall / 1e9
    kms, launches, _ = g.kernel_stats()
    adj_ms, adj_launches = g.adjoint_kernel_stats()
    support = g.source_support()
    copy_gbps = rfa.rfa_copy_bandwidth(1 << 30, 10)
    g.close()
    avg_ms = kms / max(launches, 1)
    adj_avg_ms = adj_ms / max(adj_launches, 1)
    # the perfusion factor field adds one float read per voxel-step
    fwd = roofline_dict((BYTES_PER_VOXEL_STEP + 4) * case.n_voxels + SOURCE_BYTES * support,
                        avg_ms, kernel_name(plan) + " (forward)", launches_timed=launches,
                        source_support_voxels=support)
    adj = roofline_dict(ADJ_BYTES_PER_VOXEL_STEP * case.n_voxels + ADJ_SOURCE_BYTES * support,
                        adj_avg_ms, "k_adjoint_tiled (adjoint)", launches_timed=adj_launches,
                        copy_ceiling_GBps=round(copy_gbps, 1), source_support_voxels=support)
    adj["traffic"] = traffic_record(5, ADJ_PLAN, "k_adjoint_tiled")
    # the dominant kernel (more time in the timed region) carries the roofline
    dominant, other = (adj, fwd) if adj_ms > kms else (fwd, adj)
    out = {
        "value": round(value, 3),
        "unit": "GVoxel-updates/s",
        "ms_per_step": round(wall / steps * 1e3, 3),
        "config": {"workload": f"differentiation: 9-tine umbrella 128^3 @0.5mm, {n_steps} x "
                               f"{case.dt} s, 16^3 B-spline perfusion lattice; value counts "
                               f"forward + adjoint per simulated step, checkpoint every "
                               f"{ckpt} steps with recomputation",
                   "kept_trajectory_GVox_s": round(kept_value, 3),
                   "kept_trajectory_gradients_equal": bool(np.array_equal(dP, dP_kept)),
                   "loss": loss, "dL_dP": [float(x) for x in dP],
                   "rooflines_from": "the kept-trajectory launches (same kernels and "
                                     "launch shapes; the checkpointed schedule adds the "
                                     "recompute steps)"},
        "roofline": with_traffic_rate(dominant),
        "roofline_other_kernel": with_traffic_rate(other),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_adjoint()
    return out


def cpu_baseline_adjoint() -> dict:
    """The oracle's discrete adjoint (its forward, keeping the trajectory,
    then the FP64 transpose of every step with the damage-rate derivative)
    on the differentiation workload's 32^3 copy, all host cores and one; the
    rate counts forward + adjoint per simulated voxel-step, as the GPU's
    value does.  The weights dL/dOmega are seeded random numbers (the cost
    does not depend on them)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1907_05709_amd import workloads as W
    O.build(force=False)
    case = W.case_differentiation(n=32, dx=2e-3, n_steps=600)
    q, gt, _ = O.source(case, per_tine=True)
    f = O.bspline_field(case.shape, np.zeros((16, 16, 16)))
    w = np.random.default_rng(5).standard_normal(case.shape) * 1e-3
    threads = _threads()
    res = {}
    for n_thr in (threads, 1):
        O.set_threads(n_thr)
        t0 = time.perf_counter()
        O.adjoint(case, w, q=q, perf=f)     # forward (trajectory kept), then the adjoint
        res[n_thr == 1] = time.perf_counter() - t0
    O.set_threads(threads)
    vs = case.n_voxels * case.n_steps
    return {"value": round(vs / res[False] / 1e9, 5), "unit": "GVoxel-updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"the workload's 32^3 copy at 2 mm, 600 x 0.02 s: forward + discrete "
                      f"adjoint, FP64 ({res[False]:.1f} s with {threads} threads, "
                      f"{res[True]:.1f} s with 1)",
            "single_core": {"value": round(vs / res[True] / 1e9, 5),
                            "unit": "GVoxel-updates/s", "cores": 1}}


# displacement (3 x 4) + the state's hi word (4) + output (4); lo words are
# read only for cells at or above 1024 degC and samples on a voxel centre
# (here the walls' zero-displacement voxels, under 2 %), not counted
WARP_BYTES_PER_VOXEL = 20
WARP2_BYTES_PER_VOXEL = 32  # two fields
WARP_PLAN = {"threads": 256, "tile_z": 64, "tile_y": 4, "x_voxels_per_thread": 4}
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
                                           "algorithmic_GBps": round(WARP2_BYTES_PER_VOXEL * n / (kf_ms * 1e-3) / 1e9, 1)}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_record(6, WARP_PLAN, "k_warp"),
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
