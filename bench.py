"""Benchmark of the slice-streaming Lennard-Jones path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lj_fluid_4m]
               [--serve-requests R] [--no-cpu-baseline] [--no-drift] [--quick]

One "step" is one velocity-Verlet step of the whole hot path (finalise/binning, pair
forces, integration, migration) over all slices of the workload, run inside the
persistent kernel.  Inputs are resident in HBM before the timed region starts.

Besides the timed FP32-force and FP64 legs on the 4,194,304-atom fluid, the default run
reports (each leg can be switched off):
  * the precision report: max normalised force error e_i of both modes against the FP64
    oracle on a seeded 1% subsample, at t = 0 and after the 1000-step drift run, and the
    1000-step energy drift of both modes with an OLS-slope equality test;
  * the 2048-atom fluid: 100-step drift of both GPU modes and of the oracle itself;
  * the 33,554,432-atom liquid: both modes, 1000 steps, subsample e_i at t = 0 and
    t = 1000, drift per atom-step;
  * the 8,388,608-atom slab: 2000 steps FP32 forces, per-slice counts, migrations,
    worker utilisation from the item trace;
  * the served ensemble: all 2000 Poisson requests, and a 64 MB-budget run over the
    first requests;
  * the FP64 oracle on the host cores (bounded sample) and one thread.
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
from paper_2507_11289_amd import tracecheck  # noqa: E402

METRIC = "atom-steps/s at 4M-atom LJ fluid, FP32-force vs FP64 plain; served p50/p99 latency"
FP32_PEAK = 157.3      # TFLOP/s, MI355X vector FP32 (packed) -- the figure the roofline uses
FP64_PEAK = 78.6       # TFLOP/s, MI355X vector FP64
HBM_PEAK = 8000.0      # GB/s
# the kernel and the host code that sizes its work items: both shape its memory traffic
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_11289_amd", "csrc", f)
                  for f in ("md_device.hip", "md_host.hip", "md_internal.h")]

# Counter figures of the persistent kernels on lj_fluid_4m per atom-step, from rocprofv3
# --pmc runs of this file over 100-step launches: FETCH_SIZE and WRITE_SIZE scaled by what
# the same counters read for a plain device copy of known size (0.50001 and 1.00000);
# SQ_INSTS_VALU_FLOPS_FP32/FP64 x 64 (the counter gives FLOPs per 64 lanes, read on an FP32
# multiply of known size); SQ_INSTS_VALU_MFMA_MOPS_F32 x 512.  They are reported only while
# the kernel sources have the hash they were taken on (profiles/persistent_f32_lean_lj_fluid_4m.md,
# profiles/persistent_f64_lean_lj_fluid_4m.md); otherwise null.
COUNTERS = {
    "source_sha256": "6e1a6751995e5111032a9a1963a3a853e5d5cd26b321a83a85619fcdc6d77bcf",
    "workload": "lj_fluid_4m",
    "persistent_f32_lean": {
        "hbm_read_bytes_per_atom_step": 254.1, "hbm_write_bytes_per_atom_step": 80.7,
        "valu_fp32_flop_per_atom_step": 2351.9, "valu_fp64_flop_per_atom_step": 54.5,
        "mfma_f32_flop_per_atom_step": 3773.2, "valu_instructions_per_cell_step": 1108.0,
        "valu_pipe_busy": 0.748, "l2_hit_rate": 0.36, "lds_conflict_cycles_per_lds_cycle": 1.666,
        "profile": "profiles/persistent_f32_lean_lj_fluid_4m.md"},
    "persistent_f64_lean": {
        "hbm_read_bytes_per_atom_step": 313.1, "hbm_write_bytes_per_atom_step": 65.2,
        "valu_fp32_flop_per_atom_step": 107.1, "valu_fp64_flop_per_atom_step": 3656.8,
        "mfma_f32_flop_per_atom_step": 3773.2, "valu_instructions_per_cell_step": 1704.0,
        "valu_pipe_busy": 0.571, "l2_hit_rate": 0.397, "lds_conflict_cycles_per_lds_cycle": 0.499,
        "profile": "profiles/persistent_f64_lean_lj_fluid_4m.md"},
}


def counter_report(kernel, workload, atom_steps_per_launch, launch_s):
    """Counter figures of `kernel` scaled to one launch of the timed leg: HBM bytes per
    launch, GB/s, executed FLOP/s; None when the sources or the workload differ from the
    profiled ones."""
    if not COUNTERS or COUNTERS["source_sha256"] != source_sha() or workload != COUNTERS["workload"]:
        return None
    c = COUNTERS[kernel]
    bpas = c["hbm_read_bytes_per_atom_step"] + c["hbm_write_bytes_per_atom_step"]
    per_launch = bpas * atom_steps_per_launch
    return {
        "hbm_bytes_per_launch": per_launch, "hbm_bytes_per_atom_step": bpas,
        "algorithmic_bytes_per_atom_step": 104.0, "hbm_gbs": per_launch / launch_s / 1e9,
        "frac_hbm_peak": per_launch / launch_s / 1e9 / HBM_PEAK,
        "executed_valu_fp32_tflops": c["valu_fp32_flop_per_atom_step"] * atom_steps_per_launch / launch_s / 1e12,
        "executed_valu_fp64_tflops": c["valu_fp64_flop_per_atom_step"] * atom_steps_per_launch / launch_s / 1e12,
        "executed_mfma_f32_tflops": c["mfma_f32_flop_per_atom_step"] * atom_steps_per_launch / launch_s / 1e12,
        "valu_instructions_per_cell_step": c["valu_instructions_per_cell_step"],
        "valu_pipe_busy": c["valu_pipe_busy"], "l2_hit_rate": c["l2_hit_rate"],
        "lds_conflict_cycles_per_lds_cycle": c["lds_conflict_cycles_per_lds_cycle"],
        "profile": c["profile"],
    }


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def subsample(n, frac, seed):
    """Seeded partial Fisher-Yates choice of round(frac * n) ids (sorted)."""
    m = max(1, int(round(frac * n)))
    u = inputs.Stream(seed).uniform(m)
    idx = np.arange(n, dtype=np.int64)
    for k in range(m):
        j = k + int(u[k] * (n - k))
        idx[k], idx[j] = idx[j], idx[k]
    return np.sort(idx[:m])


def ols(t, e):
    """Least-squares slope of e against t, its standard error and the RMS residual."""
    t = np.asarray(t, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    tm = t.mean()
    sxx = float(((t - tm) ** 2).sum())
    b = float(((t - tm) * (e - e.mean())).sum() / sxx)
    resid = e - (e.mean() + b * (t - tm))
    m = len(t)
    se = math.sqrt(float((resid ** 2).sum()) / max(m - 2, 1) / sxx)
    return b, se, float(np.sqrt(np.mean(resid ** 2)))


def drift_summary(t, E, n):
    """E: total energy samples at steps t; per atom: total change, OLS slope and its SE."""
    e = np.asarray(E, dtype=np.float64) / n
    b, se, rms = ols(t, e)
    return {"drift_total_per_atom": float(e[-1] - e[0]), "drift_per_atom_step": b,
            "slope_stderr": se, "sigma_E_per_atom": rms, "samples": int(len(e))}


def equal_drift(a, b):
    """Equal drift: the two OLS slopes differ by at most twice the standard error of
    their difference."""
    diff = abs(a["drift_per_atom_step"] - b["drift_per_atom_step"])
    se = math.hypot(a["slope_stderr"], b["slope_stderr"])
    return {"equal": bool(diff <= 2.0 * se), "slope_difference": diff, "stderr_of_difference": se}


def force_errors(F, ids, oracle_out):
    from oracle import ref

    e = ref.force_error(F[ids], oracle_out["F"], oracle_out["scale"])
    return {"max": float(e.max()), "median": float(np.median(e)), "atoms": int(len(ids))}


def gpu_preheat(seconds=0.5):
    """Untimed FP32 matrix products for `seconds`, before any timed leg: an idle GPU runs at
    a low clock, and the first short timed window would otherwise measure its ramp-up."""
    import torch

    a = torch.randn(4096, 4096, device="cuda")
    b = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            a = torch.mm(a, b) * 1e-3
        torch.cuda.synchronize()
    del a, b


def timed_leg(sysm, prec, steps, warmup, stream, launch_steps, schedule=None, repeats=2, preheat=0.0):
    """Load, `preheat` seconds of `gpu_preheat`, warm-up, then exactly `steps` steps in one
    md_step call bracketed by syncs (then `repeats` more such windows, for the spread only).
    Every persistent launch (warm-up and timed) covers at most `launch_steps` steps.
    `schedule`: optional (claim order, wavefront levels, XCD queues) for scheduler studies."""
    import torch

    sim = md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec)
    sim.set_stream(stream.cuda_stream)
    sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, launch_steps)
    if schedule is not None:
        order, levels, xcd = schedule
        sim.set_option(md.OPT_CLAIM_ORDER, order)
        sim.set_option(md.OPT_WAVEFRONT_LEVELS, levels)
        sim.set_option(md.OPT_XCD_QUEUES, xcd)
    sim.load(sysm.pos, sysm.vel)
    if preheat > 0:
        gpu_preheat(preheat)
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
    # the same window twice more, continuing the trajectory (for the spread only: the
    # reported throughput is the first window's)
    times = [ev_s]
    for _ in range(repeats):
        ev0.record(stream)
        sim.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) * 1e-3)
    # pair statistics at the end of the timed windows (candidates C, in-range P per atom-step)
    sim.set_option(md.OPT_COUNT_PAIRS, 1)
    sim.step(2)
    cs = sim.stats()
    C = cs.candidates / cs.counted_steps
    P = cs.in_range / cs.counted_steps
    sim.close()
    return {"wall_s": wall, "event_s": ev_s, "kernel_s": st.last_kernel_seconds,
            "launches": st.last_launches, "grid": st.persistent_grid, "chunks": st.chunks_per_slice,
            "C": C, "P": P, "repeat_event_s": times}


def run_with_samples(sysm, prec, steps, every, ids=None, oracle_t0=None, miglog=False):
    """`steps` steps with energy samples every `every`; subsample force errors at the
    start and end against the oracle (forces of the GPU's own positions at the end)."""
    from oracle import ref

    g = ref.geometry(sysm.box, sysm.slices, sysm.rc)
    out = {}
    with md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec) as sim:
        sim.set_option(md.OPT_ENERGY_EVERY, every)
        if miglog:
            sim.set_option(md.OPT_MIGRATION_LOG, 1)
        sim.load(sysm.pos, sysm.vel)
        if ids is not None:
            _, _, F0 = sim.state()
            out["force_error_t0"] = force_errors(F0, ids, oracle_t0)
            del F0
        out["slice_counts_t0"] = sim.slice_counts()
        sim.step(steps)
        st = sim.stats()
        out["ms_per_step"] = 1e3 * st.last_step_seconds / steps
        out["kernel_ms_per_step"] = 1e3 * st.last_kernel_seconds / steps
        e = sim.energy_log()
        U, K, W = sim.energy_virial()
        out["slice_counts_end"] = sim.slice_counts()
        if miglog:
            out["miglog"] = sim.migration_log()
        if ids is not None:
            pos, _, F = sim.state()
            o = ref.forces_subset(g, pos, ids)
            out["force_error_end"] = force_errors(F, ids, o)
            del pos, F
    t = np.concatenate([e[:, 0], [float(steps)]])
    E = np.concatenate([e[:, 1] + e[:, 2], [U + K]])
    out["drift"] = drift_summary(t, E, sysm.n)
    return out


def precision_and_drift_leg(sysm, steps, every=10):
    """Both modes from the same state: subsample e_i at t = 0 and at the end, drift."""
    from oracle import ref

    g = ref.geometry(sysm.box, sysm.slices, sysm.rc)
    ids = subsample(sysm.n, 0.01, 2507)
    o0 = ref.forces_subset(g, sysm.pos, ids)
    res = {"subsample": f"seeded 1% of the atoms ({len(ids)} ids), oracle forces of the GPU's own "
                        f"FP64 positions", "steps": steps, "energy_every": every}
    for name, prec in (("fp32_force", md.MD_FP32_FORCE), ("fp64", md.MD_FP64)):
        log(f"[bench] {sysm.name} {name}: {steps} steps, energy every {every}, subsample errors")
        r = run_with_samples(sysm, prec, steps, every, ids, o0)
        res[name] = {"max_e_t0": r["force_error_t0"]["max"], "median_e_t0": r["force_error_t0"]["median"],
                     f"max_e_t{steps}": r["force_error_end"]["max"],
                     f"median_e_t{steps}": r["force_error_end"]["median"],
                     "ms_per_step_with_samples": r["ms_per_step"], **r["drift"]}
    res["gate"] = {"fp32_force": 1e-5, "fp64": 1e-12}
    res["within_gate"] = bool(max(res["fp32_force"]["max_e_t0"], res["fp32_force"][f"max_e_t{steps}"]) <= 1e-5
                              and max(res["fp64"]["max_e_t0"], res["fp64"][f"max_e_t{steps}"]) <= 1e-12)
    res["equal_drift"] = equal_drift(res["fp32_force"], res["fp64"])
    return res


def small_fluid_drift_leg():
    """lj_fluid_2048, 100 steps, energy every step: both GPU modes and the oracle."""
    from oracle import ref

    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, s.rc)
    out = {}
    for name, prec in (("gpu_fp32_force", md.MD_FP32_FORCE), ("gpu_fp64", md.MD_FP64)):
        out[name] = run_with_samples(s, prec, 100, 1)["drift"]
    o = ref.run(g, s.pos, s.vel, s.dt, 100, every=1)
    out["oracle_fp64"] = drift_summary(o["elog"][:, 0], o["elog"][:, 1] + o["elog"][:, 2], s.n)
    out["equal_drift_fp32_vs_oracle"] = equal_drift(out["gpu_fp32_force"], out["oracle_fp64"])
    out["equal_drift_fp64_vs_oracle"] = equal_drift(out["gpu_fp64"], out["oracle_fp64"])
    return out


def slab_leg(steps=2000, trace_steps=100):
    """The vapour-liquid slab: throughput, per-slice counts, migrations, utilisation."""
    s = inputs.lj_slab_8m()
    log(f"[bench] lj_slab_8m: {steps} steps FP32 forces, energy every 20, migration log")
    r = run_with_samples(s, md.MD_FP32_FORCE, steps, 20, miglog=True)
    c0, c1 = r["slice_counts_t0"], r["slice_counts_end"]
    mig = r["miglog"]
    out = {"n_atoms": s.n, "slices": s.slices, "steps": steps,
           "atom_steps_per_s": s.n * steps / (r["ms_per_step"] * 1e-3 * steps),
           "ms_per_step": r["ms_per_step"], "kernel_ms_per_step": r["kernel_ms_per_step"],
           "atoms_per_slice_t0": {"min": int(c0.min()), "max": int(c0.max()), "mean": float(c0.mean())},
           "atoms_per_slice_end": {"min": int(c1.min()), "max": int(c1.max()), "mean": float(c1.mean())},
           "migrations": {"left": int(mig[:, :, 0].sum()), "right": int(mig[:, :, 1].sum()),
                          "per_step_mean": float(mig.sum() / steps),
                          "max_per_slice_step": int(mig.max())},
           "counts_conserved": bool(int(c1.sum()) == s.n), **{"drift": r["drift"]}}
    # counts at the end = counts at the start + migrations in - migrations out
    inflow = np.roll(mig[:, :, 1].sum(axis=0), 1) + np.roll(mig[:, :, 0].sum(axis=0), -1)
    out["counts_balance_migrations"] = bool((c1 == c0 + inflow - mig.sum(axis=(0, 2))).all())
    log(f"[bench] lj_slab_8m: item trace over {trace_steps} steps")
    with md.Sim(s.box, s.slices, s.rc, s.dt, md.MD_FP32_FORCE) as sim:
        sim.load(s.pos, s.vel)
        sim.step(10)
        sim.set_option(md.OPT_TRACE, 1)
        sim.step(trace_steps)
        rec, _ = sim.trace()
        st = sim.stats()
    u = tracecheck.utilisation(rec, st.persistent_grid)
    chk = tracecheck.check(rec, s.slices)
    out["utilisation"] = {"steps": trace_steps, "workers": st.persistent_grid, **u,
                          "races": len(chk["violations"])}
    return out


def system_info():
    """ROCm version and rocm-smi's clocks and power cap (whatever of it the box reports).
    Runs child processes, so it is called before anything initialises the GPU."""
    import subprocess

    env = {}
    try:
        with open("/opt/rocm/.info/version") as f:
            env["rocm"] = f.read().strip()
    except OSError:
        env["rocm"] = None
    for key, flag in (("clocks", "--showclocks"), ("power_cap", "--showmaxpower")):
        try:
            r = subprocess.run(["rocm-smi", flag, "--json"], capture_output=True, text=True, timeout=30)
            env[key] = json.loads(r.stdout) if r.returncode == 0 and r.stdout.strip() else None
        except (OSError, ValueError, subprocess.SubprocessError):
            env[key] = None
    return env


def environment(sysinfo):
    """GPU model and architecture, HIP / torch versions, plus `system_info()`."""
    import torch

    pr = torch.cuda.get_device_properties(0)
    return {"gpu": torch.cuda.get_device_name(0), "arch": getattr(pr, "gcnArchName", None),
            "compute_units": pr.multi_processor_count, "hbm_bytes": pr.total_memory,
            "torch": torch.__version__, "hip": torch.version.hip, **sysinfo}


def sampling_leg(sysm, stream, steps=200, launch_steps=100, warmup=20):
    """FP32-force ms per step with energy samples every 100 and every 10 steps (a launch runs
    all its steps in the kernel variant its sampled steps need)."""
    import torch

    out = {"steps": steps, "steps_per_launch": launch_steps}
    for every in (100, 10):
        with md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, md.MD_FP32_FORCE) as sim:
            sim.set_stream(stream.cuda_stream)
            sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, launch_steps)
            sim.set_option(md.OPT_ENERGY_EVERY, every)
            sim.load(sysm.pos, sysm.vel)
            sim.step(warmup)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sim.step(steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            out[f"every_{every}_ms_per_step"] = ev0.elapsed_time(ev1) / steps
    return out


def thermostat_leg(sysm, stream, steps=100, warmup=20):
    """Per-slice velocity-scaling thermostat (NVT) runs of `sysm` at its own temperature, both
    precisions: ms per step of one `steps`-step launch after `warmup` steps, and the kinetic
    temperature 2K / (3N - 3) at the end."""
    import torch

    out = {"steps": steps, "warmup": warmup, "T0": sysm.meta["T"]}
    for name, prec in (("fp32_force", md.MD_FP32_FORCE), ("fp64", md.MD_FP64)):
        with md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec) as sim:
            sim.set_stream(stream.cuda_stream)
            sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, steps)
            sim.set_thermostat(sysm.meta["T"])
            sim.load(sysm.pos, sysm.vel)
            sim.step(warmup)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sim.step(steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / steps
            _, K, _ = sim.energy_virial()
            out[name] = {"ms_per_step": ms, "atom_steps_per_s": sysm.n / (1e-3 * ms),
                         "T_end": 2.0 * K / (3.0 * sysm.n - 3.0)}
    return out


def serve_leg(reqs, systems, budget_bytes=96 << 30, max_runs=64, label=""):
    """Open-loop replay of the given requests (arrival times of the seeded schedule)."""
    sv = md.Server(budget_bytes, max_runs)
    tickets = {}
    drifts = []
    waits, runs = [], []  # server clock: admission wait and resident time of each run
    rejected = 0
    t_origin = time.perf_counter()
    pending = set()
    i = 0
    results = {}
    while i < len(reqs) or pending:
        now = time.perf_counter() - t_origin
        while i < len(reqs) and reqs[i].arrival <= now:
            s = systems[i]
            try:
                tickets[i] = sv.submit(s.box, s.slices, s.pos, s.vel, reqs[i].steps,
                                       precision=md.MD_FP32_FORCE, energy_every=100, tag=i)
                pending.add(i)
            except md.MDError as e:
                if e.code != md.MD_ENOMEM:
                    raise
                rejected += 1
            i += 1
        for j in list(pending):
            rc, r = sv.poll(tickets[j])
            if rc != md.MD_PENDING:
                pending.discard(j)
                results[j] = (rc, time.perf_counter() - t_origin)
                if rc == md.MD_OK:
                    drifts.append(r.drift_per_atom_step)
                    waits.append(r.t_admit - r.t_submit)
                    runs.append(r.t_done - r.t_admit)
        time.sleep(0.0005)
    t_end = time.perf_counter() - t_origin
    stats = sv.stats()
    thread_s = sv.times()
    sv.close()
    ok = [j for j, (rc, _) in results.items() if rc == md.MD_OK]
    lat = np.array([results[j][1] - reqs[j].arrival for j in ok])
    atom_steps = sum(reqs[j].n * reqs[j].steps for j in ok)
    return {
        "requests": len(reqs), "label": label, "budget_bytes": budget_bytes, "max_runs": max_runs,
        "completed": len(ok), "failed": len(results) - len(ok), "rejected_never_fit": rejected,
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "aggregate_atom_steps_per_s": atom_steps / (t_end - reqs[0].arrival),
        "offered_atom_steps_per_s": sum(r.n * r.steps for r in reqs) / max(reqs[-1].arrival, 1e-9),
        "median_drift_per_atom_step": float(np.median(drifts)) if drifts else None,
        "max_abs_drift_per_atom_step": float(np.max(np.abs(drifts))) if drifts else None,
        "launches": stats["launches"], "wall_s": t_end, "server_thread_s": thread_s,
        "p50_admission_wait_s": float(np.percentile(waits, 50)) if waits else None,
        "p99_admission_wait_s": float(np.percentile(waits, 99)) if waits else None,
        "p50_resident_s": float(np.percentile(runs, 50)) if runs else None,
        "p99_resident_s": float(np.percentile(runs, 99)) if runs else None,
    }


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sysm, budget_s=20.0):
    """The FP64 oracle, as it stands, on the host cores: a bounded number of steps of the
    bench workload with every thread; the 2048-atom fluid's full 100 steps with every
    thread and with one thread."""
    from oracle import ref

    g = ref.geometry(sysm.box, sysm.slices, sysm.rc)
    threads = ref.get_threads()
    t0 = time.perf_counter()
    ref.forces_cells(g, sysm.pos)
    one = time.perf_counter() - t0
    k = max(1, min(20, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    ref.run(g, sysm.pos, sysm.vel, sysm.dt, k)
    dt = time.perf_counter() - t0
    s0 = inputs.lj_fluid_2048()
    g0 = ref.geometry(s0.box, s0.slices, s0.rc)
    t0 = time.perf_counter()
    ref.run(g0, s0.pos, s0.vel, s0.dt, 100)
    small_all = time.perf_counter() - t0
    ref.set_threads(1)
    try:
        t0 = time.perf_counter()
        ref.run(g0, s0.pos, s0.vel, s0.dt, 100)
        small_one = time.perf_counter() - t0
    finally:
        ref.set_threads(threads)
    return {"value": sysm.n * k / dt, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{sysm.name}: {k} velocity-Verlet steps of all {sysm.n} atoms "
                      f"(+1 initial force pass), FP64, {dt:.1f} s",
            "cpu_model": cpu_model(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "lj_fluid_2048_100_steps": {"atom_steps_per_s_all_threads": s0.n * 100 / small_all,
                                        "atom_steps_per_s_one_thread": s0.n * 100 / small_one,
                                        "seconds_all_threads": small_all, "seconds_one_thread": small_one}}


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


def flop_calibration(n=1 << 28, reps=5):
    """An elementwise FP32 product of known size (n multiplies per launch), for reading the
    lane factor of the SQ_INSTS_VALU_FLOPS_FP32 counter."""
    import torch

    a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a).uniform_()
    torch.cuda.synchronize()
    for _ in range(reps):
        a.mul_(b)
    torch.cuda.synchronize()
    print(json.dumps({"fp32_multiplies_per_launch": n, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="lj_fluid_4m", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--small-budget-requests", type=int, default=300)
    ap.add_argument("--drift-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-drift", action="store_true", help="skip the precision/drift legs")
    ap.add_argument("--no-32m", action="store_true", help="skip the 33.5M-atom precision study")
    ap.add_argument("--no-slab", action="store_true", help="skip the slab leg")
    ap.add_argument("--no-thermostat", action="store_true", help="skip the thermostat (NVT) leg")
    ap.add_argument("--no-sampling", action="store_true", help="skip the energy-sampling leg")
    ap.add_argument("--quick", action="store_true",
                    help="timed legs only (no drift, 32M, slab, serving or CPU legs)")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--launch-steps", type=int, default=100,
                    help="steps per persistent launch (warm-up and timed launches alike)")
    ap.add_argument("--claim-order", choices=["dataflow", "wavefront"], default="dataflow",
                    help="scheduler of the timed legs (scheduler studies; the headline uses dataflow)")
    ap.add_argument("--wavefront-levels", type=int, default=4, help="time levels of --claim-order wavefront")
    ap.add_argument("--xcd-queues", action="store_true", help="one work queue per XCD in the timed legs")
    ap.add_argument("--flop-calibration", action="store_true",
                    help="only run an FP32 multiply of known size (counter calibration)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the slice-streaming path is built and measured "
              "on one MI355X; sharding over several GPUs is designed but not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.quick:
        args.no_drift = args.no_32m = args.no_slab = args.no_thermostat = args.no_sampling = True
        args.no_cpu_baseline = True
        args.serve_requests = args.small_budget_requests = 0
    # (child processes only before the GPU is initialised)
    sysinfo = {} if args.quick else system_info()

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.flop_calibration:
        flop_calibration()
        return
    stream = torch.cuda.Stream()
    log(f"[bench] generating {args.workload}")
    sysm = inputs.WORKLOADS[args.workload]()
    n = sysm.n
    log(f"[bench] n={n} box={sysm.box} slices={sysm.slices}")

    schedule = None
    if args.claim_order != "dataflow" or args.xcd_queues:
        schedule = (md.ORDER_WAVEFRONT if args.claim_order == "wavefront" else md.ORDER_DATAFLOW,
                    args.wavefront_levels, 1 if args.xcd_queues else 0)
    legs = {}
    for name, prec in (("fp32_force", md.MD_FP32_FORCE), ("fp64", md.MD_FP64)):
        if args.fp32_only and prec == md.MD_FP64:
            continue
        log(f"[bench] timed leg {name}: warmup {args.warmup}, steps {args.steps}")
        legs[name] = timed_leg(sysm, prec, args.steps, args.warmup, stream, args.launch_steps, schedule,
                               repeats=0 if args.quick else 2, preheat=0.0 if args.quick else 0.5)
        log(f"[bench]   {legs[name]}")

    main_leg = legs["fp32_force"]
    T = main_leg["event_s"]
    value = n * args.steps / T
    flop_per_atom_step = 8.0 * main_leg["C"] + 14.0 * main_leg["P"]
    launch_s = main_leg["kernel_s"] / max(main_leg["launches"], 1)
    steps_per_launch = args.steps / max(main_leg["launches"], 1)
    atom_steps_per_launch = n * steps_per_launch
    achieved = flop_per_atom_step * atom_steps_per_launch / launch_s / 1e12
    # HBM bytes per launch of the timed leg (from the counters' bytes per atom-step)
    counters = counter_report("persistent_f32_lean", sysm.name, atom_steps_per_launch, launch_s)
    traffic = counters["hbm_bytes_per_launch"] if counters else None
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
                   "schedule": {"claim_order": args.claim_order, "wavefront_levels": args.wavefront_levels
                                if args.claim_order == "wavefront" else None, "xcd_queues": args.xcd_queues},
                   "slices": sysm.slices, "rc": sysm.rc, "dt": sysm.dt,
                   "rho": sysm.meta.get("rho"), "T": sysm.meta.get("T"), "precision": "fp32_force",
                   "steps_per_launch": steps_per_launch},
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
            "counters": counters,
            "kernel": "persistent_f32_lean",
            "kernel_avg_ms": 1e3 * launch_s,
            "launches": main_leg["launches"],
            "steps_per_launch": steps_per_launch,
            "flop_per_atom_step": flop_per_atom_step,
            "useful_flop_per_atom_step": 22.0 * main_leg["P"],
            "unpacked_fp32_ceiling_frac": 0.5,
        },
    }
    out["repeat_ms_per_step"] = [1e3 * t / args.steps for t in main_leg["repeat_event_s"]]
    out["median_ms_per_step"] = 1e3 * float(np.median(main_leg["repeat_event_s"])) / args.steps
    if "fp64" in legs:
        f = legs["fp64"]
        v64 = n * args.steps / f["event_s"]
        a64 = (8.0 * f["C"] + 14.0 * f["P"]) * n * args.steps / f["kernel_s"] / 1e12
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * f["event_s"] / args.steps,
                       "achieved_tflops": a64, "frac_fp64_peak": a64 / FP64_PEAK,
                       "kernel": "persistent_f64_lean",
                       "counters": counter_report("persistent_f64_lean", sysm.name,
                                                  n * args.steps / max(f["launches"], 1),
                                                  f["kernel_s"] / max(f["launches"], 1))}
        out["fp32_force_speedup_vs_fp64"] = value / v64
        out["fp64"]["repeat_ms_per_step"] = [1e3 * t / args.steps for t in f["repeat_event_s"]]

    def leg(name, fn):
        try:
            out[name] = fn()
        except Exception as e:  # report the failing leg, keep the others
            out[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] leg {name} failed: {e}")

    if not args.no_drift:
        leg("precision_" + sysm.name, lambda: precision_and_drift_leg(sysm, args.drift_steps))
        log("[bench] lj_fluid_2048 drift: both GPU modes and the oracle, 100 steps")
        leg("drift_lj_fluid_2048", small_fluid_drift_leg)
    if not args.no_32m:
        def study32():
            log("[bench] generating lj_liquid_32m")
            s32 = inputs.lj_liquid_32m()
            r = precision_and_drift_leg(s32, 1000)
            r["n_atoms"] = s32.n
            return r
        leg("precision_lj_liquid_32m", study32)
    if not args.no_slab:
        leg("slab_lj_slab_8m", slab_leg)
    if not args.no_sampling:
        log("[bench] energy sampling every 100 and every 10 steps (FP32 forces)")
        leg("sampling_" + sysm.name, lambda: sampling_leg(sysm, stream))
    if not args.no_thermostat:
        log("[bench] thermostat (NVT) runs, both precisions")
        leg("thermostat_" + sysm.name, lambda: thermostat_leg(sysm, stream))
    if args.serve_requests > 0 or args.small_budget_requests > 0:
        reqs = inputs.served_ensemble()
        m = max(args.serve_requests, args.small_budget_requests)
        log(f"[bench] generating {m} served requests")
        systems = [r.system() for r in reqs[:m]]
        if args.serve_requests > 0:
            log(f"[bench] serving leg: {args.serve_requests} requests")
            leg("served", lambda: serve_leg(reqs[:args.serve_requests], systems,
                                            label="all requests, 96 GiB budget, 64 runs"))
        if args.small_budget_requests > 0:
            k = args.small_budget_requests
            log(f"[bench] serving leg, 64 MB budget: first {k} requests")
            leg("served_small_budget", lambda: serve_leg(
                reqs[:k], systems, budget_bytes=64 << 20, max_runs=8,
                label=f"first {k} requests, 64 MB budget, 8 runs (larger runs can never fit: rejected)"))
        del systems
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        leg("cpu_baseline", lambda: cpu_baseline(sysm))
    leg("environment", lambda: environment(sysinfo))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
