#!/usr/bin/env python3
"""Throughput of the truncated-Taylor propagation of noisy two-particle walks
on one MI355X.

Default workload (the batched complex64 case): 4096 realisations of two
distinguishable walkers on open chains whose sizes are drawn uniformly from
{64, 96, ..., 1024}, on-site U ~ U[0, 4], hopping noise J ~ N(1, 0.1^2),
eps = 0, dt = 0.05, Taylor tolerance 1e-7 per step, Kahan-compensated
accumulation of the terms.  One "step" is one time step of every
realisation (all Taylor terms, the FP64 norm / truncation check).

Metric: amplitude-updates/s = (stored amplitudes of all realisations) x
(steps) / (time); one update advances one amplitude by one dt.  The state
is resident in HBM before the timed region.  The same JSON line carries
  * roofline: algorithmic HBM bytes of the dominant (step) kernel per step
    (read psi + write psi once) over its duration per step, timed with HIP
    events on the kernel's stream, against the 8 TB/s HBM3E peak;
  * fp64_plain: the same workload with complex128 state at the same
    per-step tolerance, regular launches;
  * cpu_baseline: the FP64 oracle (CSR Taylor propagator) timed on a bounded
    sample of the same workload on the host cores.

The timed region replays the captured step loop (per step: one persistent
launch of the step kernel per Taylor order present in the batch, each at
its own depth, plus the FP64 finalize).  The step kernels' duration is
taken from HIP events on the plan's stream around each replay, divided by
its steps: it includes the ~7 us finalize kernel and the claim-counter
fills, so `roofline.achieved` is a slight underestimate (the rocprofv3
kernel averages under profiles/ give the kernels alone).

`roofline.traffic` is the HBM traffic per step from rocprofv3 counters,
read from the summary under profiles/ that `--profile-summary` writes; it is
reported only while the step kernel's sources hash to the value recorded
there (null otherwise).
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


# ------------------------------------------------------------ CPU baseline

def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _oracle_sample(args):
    """Propagate one realisation with the oracle, one step at a time, until
    `budget_s` seconds of propagation have passed; returns
    (amplitude-updates, propagation seconds, steps)."""
    N, J, eps, U, dt, tol, budget_s = args
    from oracle import basis as B
    from oracle import hamiltonian as Hm
    from oracle import propagate as P
    H = Hm.hamiltonian(N, 2, J, eps, U)
    psi = B.product_state(N, [N // 2 - 1, N // 2])
    steps, spent = 0, 0.0
    while spent < budget_s:
        t0 = time.perf_counter()
        psi, _, _ = P.taylor_step(H, psi, dt, tol=tol)
        spent += time.perf_counter() - t0
        steps += 1
    return N * N * steps, spent, steps


def cpu_baseline(w, budget_s: float = 10.0):
    """The FP64 oracle on a bounded sample of the workload: one realisation
    per process (one process per core, forked before the GPU is touched),
    each propagated step by step for `budget_s` seconds; the rate is the
    summed updates over the summed per-process seconds times the cores."""
    import multiprocessing as mp
    # one process per core of the host's CPU share for one GPU (16 cores,
    # whatever the affinity mask shows)
    available = host_cores()
    cores = min(available, 16)
    sizes = w.lattice_sizes()
    sample = list(range(min(cores, w.R)))
    jobs = [(int(sizes[r]),) + w.realization(r, int(sizes[r])) + (w.dt, w.tol, budget_s) for r in sample]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_sample, jobs)
    wall = time.perf_counter() - t0
    updates = sum(r[0] for r in res)
    per_proc_rate = updates / sum(r[1] for r in res)
    return {"value": per_proc_rate * cores, "unit": "amplitude-updates/s", "cores": cores,
            "cores_in_affinity_mask": available, "kind": "oracle",
            "sample": f"realisations 0..{len(sample) - 1} (N = {[int(sizes[r]) for r in sample]}), "
                      f"{sum(r[2] for r in res)} steps in total of the FP64 CSR Taylor oracle (tol {w.tol:g}), "
                      f"{budget_s:g} s of propagation per process, {cores} processes",
            "seconds": round(wall, 2)}


# ------------------------------------------------------ profile summaries

KERNEL_SOURCES = ("paper_1612_00746_amd/csrc/step2d_impl.hpp", "paper_1612_00746_amd/csrc/ctqw_internal.hpp",
                  "paper_1612_00746_amd/csrc/step2d_dispatch.hip")
# Counter summaries of the complex64 step kernel on the C3 batch, one file
# per launch shape that was profiled (the autotuner's pick varies by box).
SUMMARY = os.path.join(ROOT, "profiles", "step2d_kernel_C3_c64_kahan_wpb{wpb}.md")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shape_tag(cols_per_lane, waves_per_block, grid_waves, band_align=128, band_mode=0, row_segments=0) -> str:
    """Launch shape of the step kernel: columns per lane, waves per block,
    the waves of the (persistent) grid and the band layout."""
    return (f"cols_per_lane={cols_per_lane} waves_per_block={waves_per_block} grid_waves={grid_waves} "
            f"band_align={band_align} band_mode={band_mode} row_segments={row_segments}")


def recorded_traffic(launch, grid_waves):
    """HBM bytes per step from the committed counter summary of this launch
    shape, if it was taken on the current kernel sources."""
    try:
        text = open(SUMMARY.format(wpb=launch.get("waves_per_block", 4))).read()
    except OSError:
        return None
    keys = ("kernel-source-sha256:", "traffic-bytes:", "launch-shape:")
    fields = dict(l.split(":", 1) for l in text.splitlines() if l.startswith(keys))
    if fields.get("kernel-source-sha256", "").strip() != kernel_source_hash():
        return None
    tag = shape_tag(launch.get("cols_per_lane", 1), launch.get("waves_per_block", 4), grid_waves,
                    launch.get("band_align", 128), launch.get("band_mode", 0), launch.get("row_segments", 0))
    if fields.get("launch-shape", "").strip() != tag:
        return None
    try:
        return int(fields["traffic-bytes"].strip())
    except (KeyError, ValueError):
        return None


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def profile_summary(trace_dir, fetch_dir, write_dir, commands, out=None, cols_per_lane=1, waves_per_block=4,
                    waves_per_cu=0, band_align=128, band_mode=0, row_segments=0, persistent=1):
    """Write the step kernels' rocprofv3 summary: duration statistics from
    the kernel trace, FETCH_SIZE / WRITE_SIZE per dispatch scaled by what the
    same counters read for the 4 GiB device copy of the same run.  A step
    launches one complex64 step kernel per Taylor order present in the
    batch; per-step figures are sums over those kernels."""
    def find(d, suffix):
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith(suffix):
                    return os.path.join(root, f)
        raise FileNotFoundError(f"{suffix} under {d}")
    stats = [r for r in _rows(find(trace_dir, "kernel_stats.csv")) if "step2d_kernel<float" in r["Name"]]
    if not stats:
        raise SystemExit("no complex64 step kernel in the trace")
    grids = {int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) // 64
             for r in _rows(find(trace_dir, "kernel_trace.csv")) if "step2d_kernel<float" in r["Kernel_Name"]}
    if len(grids) != 1:
        raise SystemExit(f"step kernels launched with different grids: {sorted(grids)}")
    grid_waves = grids.pop()
    calls = {int(r["Calls"]) for r in stats}
    if len(calls) != 1:
        raise SystemExit(f"step kernels dispatched unequal times: {sorted(calls)}")
    probe_bytes = 4096 << 20

    def counter(d, name):
        rows = [r for r in _rows(find(d, "counter_collection.csv")) if r["Counter_Name"] == name]
        per = {}
        for r in rows:
            if "step2d_kernel<float" in r["Kernel_Name"]:
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        c = [float(r["Counter_Value"]) for r in rows
             if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 100000]
        if len(per) != len(stats) or not c:
            raise SystemExit(f"{name}: step kernels or copy probe dispatches missing in {d}")
        return {k: sum(v) / len(v) for k, v in per.items()}, sum(c) / len(c)
    fk, fc = counter(fetch_dir, "FETCH_SIZE")
    wk, wc = counter(write_dir, "WRITE_SIZE")
    f_scale = probe_bytes / (fc * 1024.0)
    w_scale = probe_bytes / (wc * 1024.0)
    fetch_b = sum(fk.values()) * 1024.0 * f_scale
    write_b = sum(wk.values()) * 1024.0 * w_scale
    step_ns = sum(float(r["AverageNs"]) for r in stats)
    lines = [
        "# complex64 step kernels (step2d_kernel<float, ...>)",
        "",
        "Workload: 4096 realisations of two distinguishable walkers on open chains,",
        "N uniform in {64, 96, ..., 1024}, U ~ U[0, 4], J ~ N(1, 0.1^2), dt = 0.05,",
        "Taylor tolerance 1e-7 (6 or 7 terms per realisation), complex64 with the",
        f"compensated sum; {'persistent' if persistent else 'regular'} launches, {cols_per_lane} column(s) per lane, "
        f"{waves_per_block} wave(s) per block,",
        (f"{waves_per_cu or 'all'} resident waves per CU, " if persistent else "one block per group of items, ")
        + (f"band windows on {band_align}-byte boundaries (outputs on 32-byte ones)" if band_mode
           else f"{band_align}-byte band boundaries") + ", captured step loop;",
        "adjacent Taylor orders share one launch (each item at its own order).",
        "",
        "Commands (from the repository root, TMPDIR=/tmp):",
        "",
        *[f"    {c}" for c in commands],
        "",
        "| kernel | dispatches | average | min / max | FETCH_SIZE per dispatch | WRITE_SIZE per dispatch |",
        "|---|---|---|---|---|---|",
        *[f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} ms | "
          f"{float(r['MinNs']) / 1e6:.4f} / {float(r['MaxNs']) / 1e6:.4f} ms | "
          f"{fk.get(r['Name'], float('nan')):.0f} KiB | {wk.get(r['Name'], float('nan')):.0f} KiB |"
          for r in stats],
        "",
        "| per step (sum over the step kernels) | value |",
        "|---|---|",
        f"| step kernels' duration | {step_ns / 1e6:.4f} ms |",
        f"| FETCH_SIZE of the 4 GiB copy probe | {fc:.0f} KiB (scale {f_scale:.4f}) |",
        f"| WRITE_SIZE of the 4 GiB copy probe | {wc:.0f} KiB (scale {w_scale:.4f}) |",
        f"| HBM bytes read per step | {fetch_b / 1e9:.3f} GB |",
        f"| HBM bytes written per step | {write_b / 1e9:.3f} GB |",
        "",
        f"kernel-source-sha256: {kernel_source_hash()}",
        "launch-shape: " + shape_tag(cols_per_lane, waves_per_block, grid_waves, band_align, band_mode,
                                     row_segments),
        f"traffic-bytes: {int(round(fetch_b + write_b))}",
        "",
    ]
    out = out or SUMMARY.format(wpb=waves_per_block)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print(f"wrote {out}")


def kernel_summary(out, title, workload, commands, match, trace_dir, fetch_dir=None, write_dir=None,
                   counters_dir=None, per_step_dispatches=1, algorithmic_bytes_per_step=None):
    """A rocprofv3 summary of the kernels whose name contains `match`:
    duration statistics from the kernel trace; optionally FETCH_SIZE /
    WRITE_SIZE per dispatch scaled by the same counters of the 4 GiB copy
    probe of the run (HBM bytes per step), and the average of every other
    counter found under `counters_dir` (e.g. SQ_WAVE_CYCLES, SQ_BUSY_CYCLES,
    SQ_ACTIVE_INST_VALU).  Per-step figures sum `per_step_dispatches`
    dispatches' averages."""
    def find(d, suffix):
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith(suffix):
                    return os.path.join(root, f)
        raise FileNotFoundError(f"{suffix} under {d}")
    stats = [r for r in _rows(find(trace_dir, "kernel_stats.csv")) if match in r["Name"]]
    if not stats:
        raise SystemExit(f"no kernel matching {match!r} in the trace")
    step_ns = sum(float(r["AverageNs"]) * int(r["Calls"]) for r in stats) / (
        sum(int(r["Calls"]) for r in stats) / per_step_dispatches)
    lines = [f"# {title}", "", *workload, "", "Commands (from the repository root, TMPDIR=/tmp):", "",
             *[f"    {c}" for c in commands], "",
             "| kernel | dispatches | average | min / max |", "|---|---|---|---|",
             *[f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} ms | "
               f"{float(r['MinNs']) / 1e6:.4f} / {float(r['MaxNs']) / 1e6:.4f} ms |" for r in stats], "",
             "| per step | value |", "|---|---|",
             f"| kernel time per step ({per_step_dispatches} dispatches) | {step_ns / 1e6:.4f} ms |"]
    if algorithmic_bytes_per_step:
        lines.append(f"| algorithmic bytes per step | {algorithmic_bytes_per_step / 1e9:.3f} GB |")
        lines.append(f"| algorithmic GB/s (fraction of 8 TB/s) | {algorithmic_bytes_per_step / step_ns:.1f} "
                     f"({algorithmic_bytes_per_step / step_ns / HBM_PEAK_GBS:.4f}) |")
    if fetch_dir and write_dir:
        def counter(d, name):
            rows = [r for r in _rows(find(d, "counter_collection.csv")) if r["Counter_Name"] == name]
            k = [float(r["Counter_Value"]) for r in rows if match in r["Kernel_Name"]]
            c = [float(r["Counter_Value"]) for r in rows
                 if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 100000]
            if not k or not c:
                raise SystemExit(f"{name}: kernel or copy probe dispatches missing in {d}")
            return sum(k) / len(k), sum(c) / len(c)
        fk, fc = counter(fetch_dir, "FETCH_SIZE")
        wk, wc = counter(write_dir, "WRITE_SIZE")
        probe = 4096 << 20
        fb = fk * 1024.0 * probe / (fc * 1024.0) * per_step_dispatches
        wb = wk * 1024.0 * probe / (wc * 1024.0) * per_step_dispatches
        lines += [f"| FETCH_SIZE per dispatch (copy probe: {fc:.0f} KiB for 4 GiB) | {fk:.0f} KiB |",
                  f"| WRITE_SIZE per dispatch (copy probe: {wc:.0f} KiB for 4 GiB) | {wk:.0f} KiB |",
                  f"| HBM bytes read per step | {fb / 1e9:.3f} GB |",
                  f"| HBM bytes written per step | {wb / 1e9:.3f} GB |"]
        if algorithmic_bytes_per_step:
            lines.append(f"| counted / algorithmic bytes | {(fb + wb) / algorithmic_bytes_per_step:.3f} |")
    if counters_dir:
        rows = [r for r in _rows(find(counters_dir, "counter_collection.csv")) if match in r["Kernel_Name"]]
        names = sorted({r["Counter_Name"] for r in rows})
        avg = {n: sum(float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == n) /
               max(1, sum(1 for r in rows if r["Counter_Name"] == n)) for n in names}
        lines += ["", "| counter (average per dispatch) | value |", "|---|---|",
                  *[f"| {n} | {avg[n]:.6g} |" for n in names]]
        if "SQ_ACTIVE_INST_VALU" in avg and "SQ_WAVE_CYCLES" in avg and avg["SQ_WAVE_CYCLES"] > 0:
            lines.append(f"| SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES | {avg['SQ_ACTIVE_INST_VALU'] / avg['SQ_WAVE_CYCLES']:.4f} |")
        if "SQ_BUSY_CYCLES" in avg and "SQ_WAVE_CYCLES" in avg and avg["SQ_BUSY_CYCLES"] > 0:
            lines.append(f"| SQ_WAVE_CYCLES / SQ_BUSY_CYCLES (waves resident per busy cycle) | "
                         f"{avg['SQ_WAVE_CYCLES'] / avg['SQ_BUSY_CYCLES']:.3f} |")
    lines.append("")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print(f"wrote {out}")


# ---------------------------------------------------------------- GPU side

def build_plan(w, dtype, accumulation, launch, tol):
    from paper_1612_00746_amd import Plan, make_problem
    sizes = w.lattice_sizes()
    reals = w.all_realizations()
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])
    pr, keep = make_problem(2, w.R, sizes.tolist(), w.dt, statistics=w.statistics, dtype=dtype,
                            accumulation=accumulation, taylor_tol=tol, observables=1)
    plan = Plan(pr)
    plan._keep.append(keep)
    plan.set_launch(**launch)
    plan.set_params(J, eps, U)
    plan.bind()
    sites = np.array([[n // 2 - 1, n // 2] for n in sizes], dtype=np.int32)
    plan.init_product_state(sites)
    return plan


def time_plan(plan, steps, warmup):
    """Wall time of `steps` steps and the step kernel's average duration from
    HIP events on the plan's stream.  A captured step loop is captured (for
    both starting buffers when `steps` is odd) before the timed region."""
    import torch
    plan.propagate(warmup)
    plan.set_timing(True)
    if plan.get_launch().use_graph:
        for _ in range(1 if steps % 2 == 0 else 2):
            plan.propagate(steps)
    torch.cuda.synchronize()
    plan.set_timing(True)                      # reset the counters
    t0 = time.perf_counter()
    plan.propagate(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = plan.get_timing()
    plan.set_timing(False)
    if launches != steps:
        raise RuntimeError(f"timed {launches} step kernels for {steps} steps")
    return wall, kern_ms / launches


def run_copy_probe(mib):
    """A plain device-to-device copy of `mib` MiB (torch), timed with HIP
    events, whose FETCH_SIZE / WRITE_SIZE counters scale those of the step
    kernels in a rocprofv3 counter run; beside it the library's flat copy
    and band-sweep probes on the same buffers (practical roofs for a flat
    stream and for the step kernel's access pattern).  None when mib <= 0."""
    if mib <= 0:
        return None
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    dt_copy = e0.elapsed_time(e1) * 1e-3 / 5
    out = {"bytes_read": n * 4, "bytes_written": n * 4, "gbs": round(2 * n * 4 / dt_copy / 1e9, 1),
           "frac_of_peak": round(2 * n * 4 / dt_copy / 1e9 / HBM_PEAK_GBS, 4)}
    # The library's probes on the same buffers: a flat copy of one 16-byte
    # element per thread, and the step kernel's band row sweep (1 KiB bands
    # of 1024 x 1024 complex64 grids, 8 resident waves per CU) with no
    # arithmetic: the rate the step kernel's access pattern allows.
    grid = 1024 * 1024 * 8
    if (n * 4) % grid == 0:
        from paper_1612_00746_amd import bandwidth_probe
        for key, pattern in (("flat_copy_gbs", 0), ("band_sweep_gbs", 1)):
            bandwidth_probe(src, dst, pattern)
            e0.record()
            for _ in range(5):
                bandwidth_probe(src, dst, pattern)
            e1.record()
            torch.cuda.synchronize()
            out[key] = round(2 * n * 4 / (e0.elapsed_time(e1) * 1e-3 / 5) / 1e9, 1)
    log(f"copy probe: {out}")
    del src, dst
    torch.cuda.empty_cache()
    return out


def sample_errors(w, sample, steps, runs):
    """Max-abs amplitude error after `steps` steps of the sampled
    realisations for each (dtype, tol) in `runs`, against the complex128 GPU
    path at tolerance 1e-14 (itself held to 1e-10 of the FP64 oracle by the
    tests).  Small plans of the sample alone; launch shapes do not change
    the results."""
    from paper_1612_00746_amd import Plan, make_problem
    sizes = w.lattice_sizes()
    reals = w.all_realizations(sample)
    Ns = [int(sizes[r]) for r in sample]
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])

    def final(dtype, tol):
        pr, keep = make_problem(2, len(sample), Ns, w.dt, statistics=w.statistics, dtype=dtype,
                                accumulation="kahan", taylor_tol=tol)
        p = Plan(pr)
        p._keep.append(keep)
        p.set_params(J, eps, U)
        p.bind()
        p.init_product_state(np.array([[n // 2 - 1, n // 2] for n in Ns], dtype=np.int32))
        p.propagate(steps)
        return p.state_numpy().astype(np.complex128)
    ref = final("c128", 1e-14)
    return [float(np.max(np.abs(final(dt, tol) - ref))) for dt, tol in runs]


def rk4_compare(a):
    """Runtime of the two propagators at equal per-step accuracy (the
    analogue of the paper's RK4 / Taylor comparison, Fig. 2): the batch's
    Taylor steps at dt = 0.05 with the a-priori order for tolerance 1e-7
    against RK4 (the degree-4 step) at the largest dt for which the same
    a-priori bound allows 4 terms for every realisation; both reported as
    milliseconds per unit of simulated time."""
    import torch
    from paper_1612_00746_amd import Plan, make_problem
    from workloads import C3
    w = C3("c64")
    sizes = w.lattice_sizes()
    reals = w.all_realizations()
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])
    launch = dict(cols_per_lane=2, persistent=1, waves_per_block=1, waves_per_cu=8, use_graph=1)

    def max_order(dt):
        pr, keep = make_problem(2, w.R, sizes.tolist(), dt, dtype="c64", taylor_tol=w.tol)
        p = Plan(pr)
        p._keep.append(keep)
        p.set_params(J, eps, U)
        return int(p.orders().max())
    lo, hi = 1e-4, w.dt
    for _ in range(40):   # largest dt with every a-priori order <= 4
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if max_order(mid) <= 4 else (lo, mid)
    dt_rk4 = lo
    out = {}
    for name, dt, kw in (("taylor", w.dt, dict(taylor_tol=w.tol)), ("rk4", dt_rk4, dict(method="rk4"))):
        pr, keep = make_problem(2, w.R, sizes.tolist(), dt, statistics=w.statistics, dtype="c64",
                                accumulation="kahan", observables=1, **kw)
        plan = Plan(pr)
        plan._keep.append(keep)
        plan.set_launch(**launch)
        plan.set_params(J, eps, U)
        plan.bind()
        plan.init_product_state(np.array([[n // 2 - 1, n // 2] for n in sizes], dtype=np.int32))
        wall, kern_ms = time_plan(plan, a.steps, a.warmup)
        ms = 1e3 * wall / a.steps
        out[name] = {"dt": dt, "terms": [int(plan.orders().min()), int(plan.orders().max())],
                     "ms_per_step": round(ms, 4), "ms_per_unit_time": round(ms / dt, 2)}
        del plan
        torch.cuda.empty_cache()
    out["rk4_over_taylor_time"] = round(out["rk4"]["ms_per_unit_time"] / out["taylor"]["ms_per_unit_time"], 3)
    print(json.dumps({"comparison": "RK4 (Alg. 2) vs adaptive Taylor (Alg. 3) at per-step tolerance 1e-7",
                      "workload": w.name, **out}))


def telegraph(a):
    """The batch's step with switching hopping noise (amplitude 0.1, rate 1
    per unit time: the device flips the bonds' signs and rewrites the
    hopping tables before every step) against the same batch with static
    noise, at the tuned launch shape."""
    import torch
    from workloads import C3
    w = C3("c64")
    launch = dict(cols_per_lane=2, persistent=1, waves_per_block=1, waves_per_cu=8, use_graph=1)
    out = {}
    for name, amp in (("static", 0.0), ("switching", 0.1)):
        plan = build_plan(w, "c64", "kahan", launch, w.tol)
        if amp:
            plan.set_telegraph(amp, 1.0, 7)
            plan.bind()
            sizes = w.lattice_sizes()
            plan.init_product_state(np.array([[n // 2 - 1, n // 2] for n in sizes], dtype=np.int32))
        wall, kern_ms = time_plan(plan, a.steps, a.warmup)
        out[name] = {"ms_per_step": round(1e3 * wall / a.steps, 4),
                     "terms": [int(plan.orders().min()), int(plan.orders().max())]}
        del plan
        torch.cuda.empty_cache()
    print(json.dumps({"comparison": "switching hopping noise vs static noise", "workload": w.name, **out}))


def density(a):
    """Ensemble-averaged density matrix (Eq. 2) of 1000 realisations of two
    bosons on N = 128 (D = 8256, complex64): the gather of the states and
    one Hermitian rank-1000 update.  FLOPs counted for the lower triangle:
    4 D (D + 1) R real operations (one complex multiply-add is 8); the
    matrix cores' dense FP32 peak is 157.3 TFLOP/s."""
    import torch
    from workloads import C2
    w = C2("c64")
    reals = w.all_realizations()
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])
    from paper_1612_00746_amd import Plan, make_problem
    pr, keep = make_problem(2, w.R, w.N, w.dt, statistics="boson", dtype="c64", accumulation="kahan",
                            taylor_tol=w.tol, observables=1)
    plan = Plan(pr)
    plan.set_params(J, eps, U)
    plan.bind()
    plan.init_product_state(np.array(w.start_sites(w.N), dtype=np.int32))
    plan.propagate(20)
    rho = plan.density_matrix(0)          # warm-up (rocBLAS initialisation)
    D = rho.shape[0]
    times = []
    for _ in range(max(3, a.steps // 4)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rho = plan.density_matrix(0)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    flops = 4.0 * D * (D + 1) * w.R
    tr = float(torch.trace(rho).real)
    print(json.dumps({"metric": "ensemble density matrix, TFLOP/s", "workload": "C2 shape: 1000 x two bosons, N = 128",
                      "D": D, "realisations": w.R, "ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                      "peak_fp32_mfma_tflops": 157.3, "frac": round(flops / (ms * 1e-3) / 157.3e12, 4),
                      "trace": tr}))


def autotune_launch(plan, a) -> dict:
    """Unless --no-autotune: time the launch shapes of the plan's step on
    its batch and keep the fastest (the state is overwritten: callers set
    their start state afterwards).  Returns the launch in use."""
    if not a.no_autotune:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            plan.autotune(os.path.join(td, "tune.jsonl"), steps=3)
    l = plan.get_launch()
    return {k: int(getattr(l, k)) for k in ("cols_per_lane", "waves_per_block", "persistent", "waves_per_cu",
                                            "chunked", "band_align", "band_mode", "row_segments", "use_graph")}


def density_sweep(a):
    """The paper's post-processing-rate runs (Sec. 4: the ensemble density
    matrix formed once every 10, 25, 100, 250 or 1500 of 1500 steps, 1000
    realisations) on the two-boson workload's shape: 1000 realisations, N = 128
    (D = 8256), complex64.  For each rate the run is timed with HIP events
    on the plan's stream: the whole run, and the density-matrix calls alone
    (gather + MFMA rank-1000 update + mirror); the share of the run spent
    on <rho> is reported beside the paper's ~90 % at the most frequent
    output."""
    import torch
    from paper_1612_00746_amd import Plan, make_problem
    from workloads import C2
    w = C2("c64")
    reals = w.all_realizations()
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])
    pr, keep = make_problem(2, w.R, w.N, w.dt, statistics="boson", dtype="c64", accumulation="kahan",
                            taylor_tol=w.tol, observables=1)
    plan = Plan(pr)
    plan._keep.append(keep)
    plan.set_launch(use_graph=1, row_segments=a.row_segments)
    plan.set_params(J, eps, U)
    plan.bind()
    tuned = autotune_launch(plan, a)
    total_steps = 1500
    rows = []
    plan.init_product_state(np.array(w.start_sites(w.N), dtype=np.int32))
    plan.propagate(10)
    plan.density_matrix(0)                     # warm-up of every kernel
    torch.cuda.synchronize()
    for every in (10, 25, 100, 250, 1500):
        plan.init_product_state(np.array(w.start_sites(w.N), dtype=np.int32))
        rho_ms = 0.0
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        done = 0
        n_rho = 0
        while done < total_steps:
            plan.propagate(every)
            done += every
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rho = plan.density_matrix(0)
            e1.record()
            e1.synchronize()
            rho_ms += e0.elapsed_time(e1)
            n_rho += 1
            del rho
        t1.record()
        torch.cuda.synchronize()
        run_ms = t0.elapsed_time(t1)
        rows.append({"output_every": every, "density_matrices": n_rho, "run_ms": round(run_ms, 2),
                     "rho_ms": round(rho_ms, 2), "rho_share": round(rho_ms / run_ms, 4)})
        log(f"every {every}: run {run_ms:.1f} ms, rho {rho_ms:.1f} ms ({100 * rho_ms / run_ms:.1f} %)")
    print(json.dumps({"experiment": "post-processing rate (the rates of Sec. 4)",
                      "workload": "1000 x two bosons, N = 128, D = 8256, complex64, 1500 steps of dt = 0.05",
                      "launch": tuned, "work_items": plan.work_items()[0],
                      "rates": rows,
                      "paper_context": "post-processing about 90 % of the run at frequent output, "
                                       "cublasCher > 99.3 % of that (K40, complex single)"}))
    del plan
    torch.cuda.empty_cache()


def graph(a):
    """One particle on a 128 x 128 open square lattice (q = 2, 16384
    nodes), 4096 noisy realisations (J = 1 + 0.1 N(0, 1) per bond,
    eps ~ U[-0.5, 0.5]), dt = 0.05, 10 Taylor terms per step: first the
    general-graph path (one pass per term), then the two-dimensional
    lattice path on the same noise (all terms in one pass); complex128 with
    FP64 tables, then complex64 with FP32 tables.
    The roofline fraction counts the algorithmic bytes of a step, read psi
    and write psi once (2e per node and realisation, e = 16 or 8 bytes per
    amplitude), over the step time.  The bytes the one-term passes move are
    reported beside it: per node, realisation and term the previous term (e;
    neighbours counted as cache hits), the on-site energy (f = 8 or 4 bytes
    per real), width couplings (f each), the partial sum in and out (2e)
    and the term out (e, not on the last term)."""
    import torch
    from paper_1612_00746_amd import ell_tables, graph_evolve, lattice_edges
    probe = run_copy_probe(a.copy_probe_mib)
    side, R, order, dt = 128, 4096, 10, 0.05
    n = side * side
    g = np.random.default_rng(71)
    edges = lattice_edges((side, side))
    nbr, hop = ell_tables(n, edges, 1.0 + 0.1 * g.standard_normal((R, len(edges))))
    eps = g.uniform(-0.5, 0.5, (R, n))
    width = nbr.shape[0]
    dev = "cuda"
    nbr_d = torch.from_numpy(nbr).to(dev)
    for dtype in ("c128", "c64"):
        c64 = dtype == "c64"
        rt = torch.float32 if c64 else torch.float64
        hop_d = torch.from_numpy(hop).to(dev).to(rt)
        eps_d = torch.from_numpy(eps).to(dev).to(rt)
        psi = torch.zeros((R, n), dtype=torch.complex64 if c64 else torch.complex128, device=dev)
        psi[:, n // 2 + side // 2] = 1.0
        e, f = (8, 4) if c64 else (16, 8)
        ws = torch.empty(3 * R * n * e, dtype=torch.uint8, device=dev)
        graph_evolve(nbr_d, hop_d, eps_d, psi, dt, order, max(1, a.warmup), ws)
        torch.cuda.synchronize()
        steps = max(1, a.steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph_evolve(nbr_d, hop_d, eps_d, psi, dt, order, steps, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        per_term = e + f + f * width + 2 * e + e
        moved = (order * per_term - e) * R * n
        alg = 2 * e * R * n
        norm = float(torch.linalg.vector_norm(psi[0].to(torch.complex128)).item())
        print(json.dumps({"metric": "graph walk node-updates/s", "workload": "128 x 128 lattice, 4096 realisations",
                          "dtype": dtype, "order": order, "width": width, "ms_per_step": round(ms, 4),
                          "value": R * n / (ms * 1e-3), "unit": "node-updates/s",
                          "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(alg / (ms * 1e-3) / 8e12, 4),
                                       "bytes_per_update_algorithmic": 2 * e,
                                       "bytes_per_update_moved": round(moved / (R * n), 1),
                                       "moved_GBps": round(moved / (ms * 1e-3) / 1e9, 1)},
                          "norm_r0": norm}), flush=True)
        del hop_d, eps_d, psi, ws
        torch.cuda.empty_cache()

    # The same lattice and noise through the two-dimensional lattice path:
    # all terms of a step in one pass, per-bond tables laid out per node.
    from paper_1612_00746_amd import lattice_evolve
    Jb = 1.0 + 0.1 * np.random.default_rng(71).standard_normal((R, len(edges)))
    ev = (side - 1) * side                      # bonds along y come first in the bond list
    Jy = np.zeros((R, side, side))
    Jy[:, :side - 1, :] = Jb[:, :ev].reshape(R, side - 1, side)
    Jx = np.zeros((R, side, side))
    Jx[:, :, :side - 1] = Jb[:, ev:].reshape(R, side, side - 1)
    for dtype in ("c128", "c64"):
        c64 = dtype == "c64"
        rt = torch.float32 if c64 else torch.float64
        Jx_d = torch.from_numpy(Jx).to(dev).to(rt).contiguous()
        Jy_d = torch.from_numpy(Jy).to(dev).to(rt).contiguous()
        eps_d = torch.from_numpy(eps.reshape(R, side, side)).to(dev).to(rt).contiguous()
        psi = torch.zeros((R, side, side), dtype=torch.complex64 if c64 else torch.complex128, device=dev)
        psi[:, side // 2, side // 2] = 1.0
        e, f = (8, 4) if c64 else (16, 8)
        lattice_evolve(Jx_d, Jy_d, eps_d, psi, dt, order, max(1, a.warmup))
        torch.cuda.synchronize()
        steps = max(1, a.steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lattice_evolve(Jx_d, Jy_d, eps_d, psi, dt, order, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        alg = 2 * e * R * n
        norm = float(torch.linalg.vector_norm(psi[0].to(torch.complex128)).item())
        print(json.dumps({"metric": "lattice walk node-updates/s",
                          "workload": "128 x 128 lattice, 4096 realisations (the graph line's noise)",
                          "path": "two-dimensional lattice kernel, all terms per pass", "dtype": dtype,
                          "order": order, "ms_per_step": round(ms, 4), "value": R * n / (ms * 1e-3),
                          "unit": "node-updates/s",
                          "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(alg / (ms * 1e-3) / 8e12, 4),
                                       "bytes_per_update_algorithmic": 2 * e,
                                       "bytes_per_update_with_tables": 2 * e + 3 * f,
                                       "frac_with_tables": round((2 * e + 3 * f) * R * n / (ms * 1e-3) / 8e12, 4)},
                          "copy_probe": probe, "norm_r0": norm}), flush=True)
        del Jx_d, Jy_d, eps_d, psi
        torch.cuda.empty_cache()


def three_walkers(a):
    """Three distinguishable walkers on N = 256 (64 realisations, 1.07e9
    amplitudes, nearest-neighbour U = 1, complex64): K Taylor terms chained
    per pass over the state, ceil(n / K) passes per step.  The roofline
    counts the algorithmic bytes of a step -- read psi and write psi once,
    16 B per amplitude -- over the step kernels' time; the bytes the passes
    actually move (per amplitude: the first pass reads X and writes the
    partial sum and Psi_K, 24 B; a middle pass also reads the partial sum,
    32 B; the last reads X and the partial sum and writes the state, 24 B)
    are reported beside it.  --three-form 1: the product form (each pass
    reads and writes one state, 16 B per amplitude and pass)."""
    import torch
    from paper_1612_00746_amd import Plan, make_problem
    from workloads import C5
    w = C5()
    probe = run_copy_probe(a.copy_probe_mib)
    sizes = w.lattice_sizes()
    reals = w.all_realizations()
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals])
    pr, keep = make_problem(3, w.R, int(sizes[0]), w.dt, statistics=w.statistics, interaction=w.interaction,
                            dtype="c64", accumulation="kahan", taylor_tol=w.tol, observables=1)
    plan = Plan(pr)
    plan._keep.append(keep)
    plan.set_launch(use_graph=1, terms_per_pass=a.terms_per_pass, three_form=a.three_form)
    plan.set_params(J, eps, U)
    plan.bind()
    plan.init_product_state(np.array([w.start_sites(int(n)) for n in sizes], dtype=np.int32))
    wall, kern_ms = time_plan(plan, a.steps, a.warmup)
    amps = int(np.sum(sizes.astype(np.int64) ** 3))
    n = int(plan.orders().max())
    K = plan.get_launch().terms_per_pass or 3
    passes = -(-n // K)
    form = plan.get_launch().three_form
    if passes == 1 or form == 1:
        impl_bytes = 16.0 * passes
    else:
        impl_bytes = 24.0 + 32.0 * (passes - 2) + 24.0
    achieved = amps * 16.0 / (kern_ms * 1e-3) / 1e9
    st = plan.stats()
    print(json.dumps({
        "metric": "amplitude-updates/s per Taylor step", "value": amps * a.steps / wall,
        "unit": "amplitude-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * wall / a.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic (seeded noise draws, no dataset)",
        "config": {"workload": w.name, "realisations": w.R, "sites": int(sizes[0]), "particles": 3,
                   "amplitudes": amps, "dt": w.dt, "taylor_tol": w.tol, "taylor_order": n,
                   "terms_per_pass": K, "passes": passes,
                   "pass_form": "product of root factors" if form == 1 else "chained Taylor sum"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "step3c_kernel",
                     "kernel_ms": round(kern_ms, 4), "bytes_per_update_algorithmic": 16,
                     "bytes_per_update_moved": impl_bytes,
                     "moved_GBps": round(amps * impl_bytes / (kern_ms * 1e-3) / 1e9, 1)},
        "norm_range": [st.min_norm, st.max_norm],
        "copy_probe": probe,
    }))
    del plan
    torch.cuda.empty_cache()


def adjoint(a):
    """Seconds per gradient of the gradient workload: two bosons on N = 256,
    U = 1, 512 realisations, loss = probability that both are in nodes
    192..255 after 400 steps of dt = 0.05, gradients with respect to the 255
    baseline hoppings and 256 on-site energies, checkpoints every 32 steps
    (the forward run with checkpoints, then the adjoint: recomputation of
    each segment and the Horner recursion with the FP64 contractions);
    complex64 and complex128.  Timed with HIP events on the plan's stream
    around the whole gradient call, after one untimed gradient."""
    import torch
    from paper_1612_00746_amd import Plan, make_problem
    from workloads import C4
    for dtype in a.adjoint_dtypes.split(","):
        w = C4(dtype)
        reals = w.all_realizations()
        J = np.concatenate([r[1] for r in reals])
        eps = np.concatenate([r[2] for r in reals])
        U = np.array([r[3] for r in reals])
        pr, keep = make_problem(2, w.R, w.N, w.dt, statistics="boson", dtype=dtype, taylor_tol=w.tol)
        plan = Plan(pr)
        plan._keep.append(keep)
        plan.set_launch(row_segments=a.row_segments)
        plan.set_params(J, eps, U)
        plan.bind()
        tuned = autotune_launch(plan, a)
        sw = (np.arange(w.N) >= 192).astype(float)
        times = []
        for k in range(3):
            plan.init_product_state(list(w.start))
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            loss, gJ, gE = plan.gradient(w.n_steps, 32, sw, "product")
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            if k:
                times.append(e0.elapsed_time(e1) * 1e-3)
        sec = float(np.median(times))
        amps = w.R * w.N * (w.N + 1) // 2
        print(json.dumps({"metric": "seconds per gradient", "value": round(sec, 4), "unit": "s",
                          "higher_is_better": False, "dtype": dtype,
                          "config": {"workload": w.name, "realisations": w.R, "sites": w.N, "steps": w.n_steps,
                                     "checkpoint_every": 32, "taylor_order": int(plan.orders().max()),
                                     "amplitudes": amps, "launch": tuned,
                                     "work_items": plan.work_items()[0]},
                          "loss": loss, "grad_norm": float(np.linalg.norm(np.concatenate([gJ, gE]))),
                          "forward_equivalent_steps_per_s": round(w.n_steps / sec, 1)}), flush=True)
        del plan
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cols-per-lane", type=int, default=1)
    ap.add_argument("--accumulation", default="kahan")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--copy-probe-mib", type=int, default=4096,
                    help="device copies of this size (torch, and the library's flat and band-sweep probes), timed as practical HBM roofs (0: skip)")
    ap.add_argument("--regular", action="store_true", help="one block per item group instead of the persistent grid")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep --cols-per-lane, --waves-per-block and --waves-per-cu")
    ap.add_argument("--waves-per-block", type=int, default=4)
    ap.add_argument("--waves-per-cu", type=int, default=0, help="persistent grid: resident waves per CU (0: all)")
    ap.add_argument("--band-align", type=int, default=128, help="column-band alignment in bytes (with --no-autotune)")
    ap.add_argument("--band-mode", type=int, default=0,
                    help="0: band boundaries aligned; 1: band windows aligned (with --no-autotune)")
    ap.add_argument("--row-segments", type=int, default=0,
                    help="two particles: 0 splits few bands' rows, 1 never, k at most k segments (with --no-autotune)")
    ap.add_argument("--profile-summary", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the step kernel's rocprofv3 summary under profiles/ and exit")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line recorded in the profile summary (repeatable)")
    ap.add_argument("--kernel-summary", metavar="OUT",
                    help="write a rocprofv3 summary of the kernels matching --match to OUT and exit")
    ap.add_argument("--match", default="", help="kernel-name substring for --kernel-summary")
    ap.add_argument("--title", default="", help="title of the --kernel-summary")
    ap.add_argument("--workload-line", action="append", default=[], help="workload description line (repeatable)")
    ap.add_argument("--trace-dir", help="--kernel-summary: rocprofv3 --kernel-trace --stats output directory")
    ap.add_argument("--fetch-dir", help="--kernel-summary: rocprofv3 --pmc FETCH_SIZE output directory")
    ap.add_argument("--write-dir", help="--kernel-summary: rocprofv3 --pmc WRITE_SIZE output directory")
    ap.add_argument("--counters-dir", help="--kernel-summary: rocprofv3 --pmc output with other counters")
    ap.add_argument("--per-step", type=int, default=1, help="--kernel-summary: matching dispatches per step")
    ap.add_argument("--alg-bytes", type=float, default=0.0, help="--kernel-summary: algorithmic bytes per step")
    ap.add_argument("--rk4-compare", action="store_true",
                    help="time Alg. 2 (RK4) against the adaptive Taylor step at equal per-step accuracy on the batch")
    ap.add_argument("--density-sweep", action="store_true",
                    help="the post-processing-rate experiment: <rho> every 10 ... 1500 of 1500 steps")
    ap.add_argument("--graph", action="store_true",
                    help="time one particle on a 128 x 128 lattice, 4096 realisations (complex128)")
    ap.add_argument("--telegraph", action="store_true",
                    help="time the batch with switching hopping noise (a = 0.1, rate 1) against static noise")
    ap.add_argument("--density", action="store_true",
                    help="time the ensemble density matrix of 1000 two-boson states on N = 128 (complex64)")
    ap.add_argument("--three-walkers", action="store_true",
                    help="time the three-walker path instead (64 x 256^3 amplitudes, complex64)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time one gradient of the gradient workload (512 x two bosons, N = 256, 400 steps)")
    ap.add_argument("--adjoint-dtypes", default="c64,c128", help="--adjoint: comma-separated state types")
    ap.add_argument("--three-form", type=int, default=1,
                    help="three walkers: 0 chained Taylor sum per pass, 1 product of the polynomial's root factors")
    ap.add_argument("--terms-per-pass", type=int, default=0,
                    help="three walkers: Taylor terms chained per pass (0: the library's default)")
    a = ap.parse_args()
    if a.profile_summary:
        profile_summary(*a.profile_summary, commands=a.profile_command, cols_per_lane=a.cols_per_lane,
                        waves_per_block=a.waves_per_block, waves_per_cu=a.waves_per_cu, band_align=a.band_align,
                        band_mode=a.band_mode, row_segments=a.row_segments, persistent=0 if a.regular else 1)
        return
    if a.kernel_summary:
        kernel_summary(a.kernel_summary, a.title or a.match, a.workload_line, a.profile_command, a.match,
                       a.trace_dir, a.fetch_dir, a.write_dir, a.counters_dir, a.per_step, a.alg_bytes or None)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: realisations are independent, and a multi-GPU run would "
              "shard them with one all-reduce of the FP64 observables; only --gpus 1 is built.",
              file=sys.stderr)
        sys.exit(2)

    if a.three_walkers:
        three_walkers(a)
        return
    if a.adjoint:
        adjoint(a)
        return
    if a.rk4_compare:
        rk4_compare(a)
        return
    if a.density:
        density(a)
        return
    if a.density_sweep:
        density_sweep(a)
        return
    if a.graph:
        graph(a)
        return
    if a.telegraph:
        telegraph(a)
        return

    from workloads import C3
    w = C3("c64")
    log("cpu baseline (oracle) ..." if not a.no_cpu else "cpu baseline skipped")
    cpu = None if a.no_cpu else cpu_baseline(w, a.cpu_budget)   # before the GPU is touched
    if cpu:
        log(f"cpu baseline: {cpu['value']:.3e} updates/s on {cpu['cores']} cores ({cpu['seconds']} s)")

    import torch
    copy_probe = run_copy_probe(a.copy_probe_mib)
    sizes = w.lattice_sizes()
    amps = int(np.sum(sizes.astype(np.int64) ** 2))
    launch = {"cols_per_lane": a.cols_per_lane, "persistent": 0 if a.regular else 1,
              "waves_per_block": a.waves_per_block, "waves_per_cu": a.waves_per_cu, "use_graph": 1,
              "band_align": a.band_align, "band_mode": a.band_mode, "row_segments": a.row_segments}
    log("building the complex64 plan ...")
    plan = build_plan(w, "c64", a.accumulation, launch, w.tol)
    tuned = None
    if not a.no_autotune:
        # The autotuner times every launch shape on this batch.  The batch's
        # launch form stays persistent with the captured step loop (the
        # workload is defined with one persistent launch per step): the
        # fastest persistent candidate of the autotuner's trace is taken
        # (the fastest overall is reported beside it).  The state is
        # overwritten by tuning: start again after it.
        import tempfile
        keys = ("cols_per_lane", "waves_per_block", "persistent", "waves_per_cu", "chunked", "band_align",
                "band_mode", "row_segments")
        with tempfile.TemporaryDirectory() as td:
            trace = os.path.join(td, "trace.jsonl")
            old_trace = os.environ.get("CTQW_TUNE_TRACE")
            os.environ["CTQW_TUNE_TRACE"] = trace
            try:
                best, best_ms = plan.autotune(os.path.join(td, "tune.jsonl"), steps=3)
            finally:
                if old_trace is None:
                    del os.environ["CTQW_TUNE_TRACE"]
                else:
                    os.environ["CTQW_TUNE_TRACE"] = old_trace
            cands = [json.loads(line) for line in open(trace)] if os.path.exists(trace) else []
        tuned = {k: int(getattr(best, k)) for k in keys}
        tuned["ms"] = round(best_ms, 4)
        log(f"autotune: {tuned}")
        form = 0 if a.regular else 1
        pick = min((c for c in cands if c["ms"] > 0 and c["persistent"] == form), key=lambda c: c["ms"], default=None)
        if pick is None:
            pick = dict(tuned, persistent=form)
        log(f"launch form {'regular' if a.regular else 'persistent'}: fastest candidate "
            f"{ {k: pick[k] for k in keys} } at {pick['ms']:.4f} ms")
        launch = {k: int(pick[k]) for k in keys}
        launch["use_graph"] = 1
        plan.set_launch(**launch)
        plan.bind()
        sizes0 = w.lattice_sizes()
        plan.init_product_state(np.array([[n // 2 - 1, n // 2] for n in sizes0], dtype=np.int32))
    log("timing complex64 ...")
    wall, kern_ms = time_plan(plan, a.steps, a.warmup)
    log(f"complex64: {1e3 * wall / a.steps:.3f} ms/step, kernel {kern_ms:.3f} ms")
    st = plan.stats()
    ms_per_step = 1e3 * wall / a.steps
    updates = amps * a.steps / wall
    bytes_per_launch = amps * 16.0
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    orders = plan.orders()
    items, grid_waves = plan.work_items()
    traffic = recorded_traffic(launch, grid_waves)
    del plan
    torch.cuda.empty_cache()

    fp64 = None
    if not a.no_fp64:
        # Equal accuracy: the complex128 comparator runs at the loosest
        # tolerance whose measured error on a sample of the batch (the
        # smallest and largest chains and two more, 50 steps) is at most the
        # complex64 path's on the same sample.
        g = np.random.default_rng(5)
        sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *g.choice(w.R, 2, replace=False).tolist()})
        cands = [1e-4, 1e-5, 1e-6, 1e-7, 1e-8]
        errs = sample_errors(w, sample, 50, [("c64", w.tol)] + [("c128", t) for t in cands])
        e32, e64s = errs[0], dict(zip(cands, errs[1:]))
        tol64 = next((t for t in cands if e64s[t] <= e32), cands[-1])
        log(f"equal accuracy: c64 error {e32:.2e}; c128 errors {e64s} -> tol {tol64:g}")
        log("building the complex128 plan ...")
        p64 = build_plan(w, "c128", "plain", {"cols_per_lane": 1, "persistent": 0, "waves_per_block": 4}, tol64)
        wall64, kern64 = time_plan(p64, max(2, a.steps // 2), 2)
        log(f"complex128: kernel {kern64:.3f} ms")
        s64 = max(2, a.steps // 2)
        fp64 = {"value": amps * s64 / wall64, "unit": "amplitude-updates/s", "dtype": "c128",
                "ms_per_step": round(1e3 * wall64 / s64, 4),
                "kernel_ms": round(kern64, 4),
                "hbm_gbs_algorithmic": round(amps * 32.0 / (kern64 * 1e-3) / 1e9, 1),
                "taylor_tol": tol64,
                "taylor_order": [int(p64.orders().min()), int(p64.orders().max())],
                "launch": "regular, one per Taylor order and step",
                "equal_accuracy": {"sample": sample, "steps": 50, "reference": "complex128 GPU path at tol 1e-14",
                                   "c64_max_abs_err": e32, "c128_max_abs_err": e64s[tol64],
                                   "c128_err_by_tol": {f"{t:g}": e for t, e in e64s.items()}}}
        del p64
        torch.cuda.empty_cache()

    line = {
        "metric": "amplitude-updates/s per Taylor step",
        "value": updates,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded noise draws, no dataset)",
        "config": {"workload": w.name, "realisations": w.R, "sites": "U{64,96,...,1024}",
                   "particles": 2, "amplitudes": amps, "dt": w.dt, "taylor_tol": w.tol,
                   "taylor_order": [int(orders.min()), int(orders.max())],
                   "accumulation": a.accumulation, "launch": launch, "work_items": items},
        "hbm_gbs_algorithmic": round(updates * 16.0 / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "step2d_kernel", "kernel_ms": round(kern_ms, 4)},
        "fp64_plain": fp64,
        "speedup_fp32_batched_vs_fp64_plain": (round(updates / fp64["value"], 3) if fp64 else None),
        "norm_range": [st.min_norm, st.max_norm],
        "cpu_baseline": cpu,
        "copy_probe": copy_probe,
        # the step kernel's rate against the band row sweep with no
        # arithmetic, measured in this run (its access pattern's practical roof)
        "frac_of_band_sweep": (round(achieved / copy_probe["band_sweep_gbs"], 4)
                               if copy_probe and copy_probe.get("band_sweep_gbs") else None),
        "autotune": tuned,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
