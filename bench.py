"""Benchmark of the slice-streaming Lennard-Jones path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lj_fluid_4m]
               [--serve-requests R] [--no-cpu-baseline] [--no-drift]

One "step" is one velocity-Verlet step of the whole hot path (binning/finalise,
pair forces, integration, migration) over all slices of the workload, run inside
the persistent kernel.  Inputs are resident in HBM before the timed region starts.
Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2507_11289_amd import inputs  # noqa: E402
from paper_2507_11289_amd import md  # noqa: E402

METRIC = "atom-steps/s at 4M-atom LJ fluid, FP32-force vs FP64 plain; served p50/p99 latency"
FP32_PEAK = 157.3      # TFLOP/s, MI355X vector FP32 (packed) -- the figure the roofline uses
FP64_PEAK = 78.6       # TFLOP/s, MI355X vector FP64
HBM_PEAK = 8000.0      # GB/s
# the kernel and the host code that sizes its work items: both shape its memory traffic
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_11289_amd", "csrc", f) for f in ("md_device.hip", "md_host.hip")]

# HBM traffic of one 100-step launch of the FP32-force persistent kernel on lj_fluid_4m,
# from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) and the same
# counters on a plain device copy of known size (profiles/persistent_f32_lean_lj_fluid_4m.md).
# Valid only for the kernel and host sources they were taken on (sha256 below); otherwise null.
TRAFFIC = {
    "source_sha256": "e7c4eafbca2018a9c9ac180a1c470ab265840b6a03b37b987dd873dbac06d807",
    "workload": "lj_fluid_4m",
    "steps_per_launch": 100,
    "fetch_kib_per_launch": 68517034,      # FETCH_SIZE, mean of 3 dispatches
    "write_kib_per_launch": 26019627,      # WRITE_SIZE, mean of 3 dispatches
    "copy_fetch_factor": 0.50001,          # FETCH_SIZE KiB / KiB really read by a 1 GiB copy
    "copy_write_factor": 1.00000,          # WRITE_SIZE KiB / KiB really written by it
    "hbm_bytes_per_launch": 1.6696e+11,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def timed_leg(sysm, prec, steps, warmup, stream, launch_steps):
    """Warm-up, then exactly `steps` steps in one md_step call bracketed by syncs.
    Every persistent launch (warm-up and timed) covers `launch_steps` steps."""
    import torch

    sim = md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec)
    sim.set_stream(stream.cuda_stream)
    sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, launch_steps)
    sim.load(sysm.pos, sysm.vel)
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.stats()
    ev_s = ev0.elapsed_time(ev1) * 1e-3
    # pair statistics at the end of the timed window (candidates C, in-range P per atom-step)
    sim.set_option(md.OPT_COUNT_PAIRS, 1)
    sim.step(2)
    cs = sim.stats()
    C = cs.candidates / cs.counted_steps
    P = cs.in_range / cs.counted_steps
    sim.close()
    return {
        "wall_s": wall, "event_s": ev_s, "kernel_s": st.last_kernel_seconds,
        "launches": st.last_launches, "grid": st.persistent_grid, "chunks": st.chunks_per_slice,
        "C": C, "P": P,
    }


def drift_leg(sysm, prec, steps, every=10):
    sim = md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec)
    sim.set_option(md.OPT_ENERGY_EVERY, every)
    sim.load(sysm.pos, sysm.vel)
    sim.step(steps)
    e = sim.energy_log()
    U, K, W = sim.energy_virial()
    sim.close()
    t = np.concatenate([e[:, 0], [float(steps)]])
    E = np.concatenate([e[:, 1] + e[:, 2], [U + K]]) / sysm.n
    slope, icpt = np.polyfit(t, E, 1)
    resid = E - (slope * t + icpt)
    return {"drift_total": float(E[-1] - E[0]), "drift_per_atom_step": float(slope),
            "sigma_E": float(np.sqrt(np.mean(resid ** 2))), "samples": int(len(t))}


def cpu_baseline(sysm, budget_s=20.0):
    """The FP64 oracle, as it stands, on the host cores: a bounded number of steps."""
    from oracle import ref

    g = ref.geometry(sysm.box, sysm.slices, sysm.rc)
    t0 = time.perf_counter()
    ref.forces_cells(g, sysm.pos)
    one = time.perf_counter() - t0
    k = max(1, min(20, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    ref.run(g, sysm.pos, sysm.vel, sysm.dt, k)
    dt = time.perf_counter() - t0
    return {"value": sysm.n * k / dt, "unit": "atom-steps/s", "cores": ref.get_threads(),
            "kind": "oracle",
            "sample": f"{sysm.name}: {k} velocity-Verlet steps of all {sysm.n} atoms "
                      f"(+1 initial force pass), FP64, {dt:.1f} s"}


def serve_leg(nreq, budget_bytes=96 << 30, max_runs=64):
    """Open-loop replay of the first `nreq` requests of the served ensemble."""
    reqs = inputs.served_ensemble()[:nreq]
    systems = [r.system() for r in reqs]
    sv = md.Server(budget_bytes, max_runs)
    tickets = {}
    lat = []
    atom_steps = 0
    drifts = []
    t_origin = time.perf_counter()
    pending = set()
    i = 0
    results = {}
    while i < len(reqs) or pending:
        now = time.perf_counter() - t_origin
        while i < len(reqs) and reqs[i].arrival <= now:
            s = systems[i]
            tickets[i] = sv.submit(s.box, s.slices, s.pos, s.vel, reqs[i].steps,
                                   precision=md.MD_FP32_FORCE, energy_every=100, tag=i)
            pending.add(i)
            i += 1
        for j in list(pending):
            rc, r = sv.poll(tickets[j])
            if rc != md.MD_PENDING:
                pending.discard(j)
                results[j] = (rc, time.perf_counter() - t_origin)
                if rc == md.MD_OK:
                    drifts.append(r.drift_per_atom_step)
        time.sleep(0.0005)
    t_end = time.perf_counter() - t_origin
    stats = sv.stats()
    sv.close()
    ok = [j for j, (rc, _) in results.items() if rc == md.MD_OK]
    for j in ok:
        lat.append(results[j][1] - reqs[j].arrival)
        atom_steps += reqs[j].n * reqs[j].steps
    lat = np.array(lat)
    return {
        "requests": nreq, "completed": len(ok), "failed": len(results) - len(ok),
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "aggregate_atom_steps_per_s": atom_steps / (t_end - reqs[0].arrival),
        "offered_atom_steps_per_s": sum(r.n * r.steps for r in reqs) / max(reqs[-1].arrival, 1e-9),
        "median_drift_per_atom_step": float(np.median(drifts)) if drifts else None,
        "launches": stats["launches"],
    }


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="lj_fluid_4m", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--drift-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-drift", action="store_true")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--launch-steps", type=int, default=100,
                    help="steps per persistent launch (warm-up and timed launches alike)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the slice-streaming path is built and measured "
              "on one MI355X; multi-GPU sharding is described in DESIGN.md but not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    stream = torch.cuda.Stream()
    log(f"[bench] generating {args.workload}")
    sysm = inputs.WORKLOADS[args.workload]()
    n = sysm.n
    log(f"[bench] n={n} box={sysm.box} slices={sysm.slices}")

    legs = {}
    for name, prec in (("fp32_force", md.MD_FP32_FORCE), ("fp64", md.MD_FP64)):
        if args.fp32_only and prec == md.MD_FP64:
            continue
        log(f"[bench] timed leg {name}: warmup {args.warmup}, steps {args.steps}")
        legs[name] = timed_leg(sysm, prec, args.steps, args.warmup, stream, args.launch_steps)
        log(f"[bench]   {legs[name]}")

    main_leg = legs["fp32_force"]
    T = main_leg["event_s"]
    value = n * args.steps / T
    flop_per_atom_step = 8.0 * main_leg["C"] + 14.0 * main_leg["P"]
    launch_s = main_leg["kernel_s"] / max(main_leg["launches"], 1)
    steps_per_launch = args.steps / max(main_leg["launches"], 1)
    achieved = flop_per_atom_step * n * steps_per_launch / launch_s / 1e12
    traffic = None          # measured HBM GB/s of the dominant kernel (rocprofv3 counters)
    traffic_detail = None
    if (TRAFFIC and TRAFFIC["source_sha256"] == source_sha() and sysm.name == TRAFFIC["workload"]
            and int(steps_per_launch) == TRAFFIC["steps_per_launch"]):
        hbm_bytes = TRAFFIC["hbm_bytes_per_launch"]
        traffic = hbm_bytes / launch_s / 1e9
        traffic_detail = {"unit": "GB/s", "hbm_bytes_per_launch": hbm_bytes,
                          "frac_hbm_peak": traffic / HBM_PEAK,
                          "bytes_per_atom_step": hbm_bytes / (n * steps_per_launch),
                          "algorithmic_bytes_per_atom_step": 104.0}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair forces / f64 state, integrator and sums",
        "data": "synthetic",
        "config": {"workload": sysm.name, "n_atoms": n, "box": list(sysm.box),
                   "slices": sysm.slices, "rc": sysm.rc, "dt": sysm.dt,
                   "rho": sysm.meta.get("rho"), "T": sysm.meta.get("T"), "precision": "fp32_force",
                   "steps_per_launch": args.launch_steps},
        "pair_interactions_per_s": main_leg["P"] * n * args.steps / T,
        "candidates_per_atom": main_leg["C"],
        "in_range_per_atom": main_leg["P"],
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK,
            "traffic": traffic,
            "traffic_detail": traffic_detail,
            "kernel": "persistent_f32_lean",
            "kernel_avg_ms": 1e3 * launch_s,
            "launches": main_leg["launches"],
            "steps_per_launch": steps_per_launch,
            "flop_per_atom_step": flop_per_atom_step,
        },
    }
    if "fp64" in legs:
        f = legs["fp64"]
        v64 = n * args.steps / f["event_s"]
        a64 = (8.0 * f["C"] + 14.0 * f["P"]) * n * args.steps / f["kernel_s"] / 1e12
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * f["event_s"] / args.steps,
                       "achieved_tflops": a64, "frac_fp64_peak": a64 / FP64_PEAK}
        out["fp32_force_speedup_vs_fp64"] = value / v64
    if not args.no_drift:
        d = {}
        for name, prec in (("fp32_force", md.MD_FP32_FORCE), ("fp64", md.MD_FP64)):
            if name in legs:
                log(f"[bench] drift leg {name}: {args.drift_steps} steps, energy every 10")
                d[name] = drift_leg(sysm, prec, args.drift_steps)
        if len(d) == 2:
            a, b = d["fp32_force"], d["fp64"]
            d["equal_drift"] = abs(a["drift_total"] - b["drift_total"]) <= max(
                3 * b["sigma_E"], 0.1 * abs(b["drift_total"]))
        out["drift"] = d
    if args.serve_requests > 0:
        log(f"[bench] serving leg: {args.serve_requests} requests")
        out["served"] = serve_leg(args.serve_requests)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sysm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
