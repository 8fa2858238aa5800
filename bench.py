"""Benchmark of the MI355X Monte Carlo tracker.

One step = one complete run of the hot path (source sampling, event-based
tracking with census steps, track-length tallies, batch statistics) over the
workload below, inputs resident on the GPU.  Prints ONE JSON line.

Workload (single GPU): the pulsed slab -- one group, Sigma_t = 1, c = 0.9,
v = 1, 40 mean free paths, isotropic pulse at the centre at t = 0,
50 spatial x 100 time tally bins over [0, 20], 1e7 histories, FP64.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--algorithm event|history] [--histories N] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "histories/sec + figure of merit 1/(σ²T), plain analog vs learned-WW, 1×MI355X"
WORKLOAD = ("pulsed slab: 1 group, Sigma_t=1, c=0.9, v=1, 40 mfp, isotropic centre pulse at t=0, "
            "50 x-bins x 100 time bins on [0,20], 1e7 histories, FP64")
HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane operations per
# second (the non-packed vector rate; MI355X's 78.6 TFLOP/s FP64 counts an
# FMA as two)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_event_pulsed_slab_1e7_counters.json")
LATTICE_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_event_lattice_1e8_counters.json")
KERNEL_SOURCES = ["paper_2305_07636_amd/csrc/k_event.hip", "paper_2305_07636_amd/csrc/k_common.hpp",
                  "paper_2305_07636_amd/csrc/mcdc_internal.hpp", "paper_2305_07636_amd/build.py"]
T_START = time.perf_counter()


def log(msg):
    """Progress to stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f}s] {msg}", file=sys.stderr, flush=True)


def cpu_worker(args):
    """Run a contiguous history range of the job through the oracle."""
    first, count, N, seed = args
    import oracle
    import workloads as w

    prob = w.cfg2_slab_pulse()
    t0 = time.perf_counter()
    oracle.run(prob, N, seed, first=first, count=count)
    return time.perf_counter() - t0


def host_cpu():
    """The host CPU as lscpu reports it, and what this process may use (one
    GPU's share of the host: at most 16 worker processes)."""
    import subprocess

    info = {"os_cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        keep = ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)",
                "CPU max MHz", "L3 cache")
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in keep:
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(N, seed, target_s=15.0):
    """The oracle as it stands, on the host cores, over a bounded sample of
    the same job (histories 0..n-1), in independent processes over
    contiguous history ranges (skip-ahead makes them independent)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import oracle

    oracle.build()
    # one GPU's share of the host: 16 worker processes at most
    cores = min(16, len(os.sched_getaffinity(0)) or 1)
    # calibrate the per-core rate on a short range
    t = cpu_worker((0, 20000, N, seed))
    rate1 = 20000 / t
    per = max(1000, int(rate1 * target_s / 2))
    per = min(per, N // cores)       # the sample stays inside the job
    n = per * cores
    # a worker that dies raises BrokenProcessPool here instead of hanging
    with ProcessPoolExecutor(cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(cpu_worker, [(0, 1000, N, seed)] * cores))    # start the workers
        t0 = time.perf_counter()
        list(ex.map(cpu_worker, [(j * per, per, N, seed) for j in range(cores)]))
        wall = time.perf_counter() - t0
    return {
        "value": n / wall, "unit": "histories/s", "cores": cores, "kind": "oracle", "host": host_cpu(),
        "sample": f"histories 0..{n - 1} of the {N:.0e}-history job, {cores} processes x {per} "
                  f"contiguous histories, serial C oracle (gcc -O2, no contraction), wall {wall:.1f} s",
        "single_core_histories_per_s": rate1,
    }


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(path, histories):
    """Per-launch hardware counters of the event form's step kernel
    (k_event) from a committed rocprofv3 summary: calibrated HBM bytes
    (FETCH_SIZE, WRITE_SIZE) and VALU instructions per event.  None if the
    kernel sources changed since, or the summary is of another size."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("histories") != histories:
        return None
    return rec


def atomic_ceiling(n_bins, n_ops=1 << 27):
    """FP64 atomic adds per second that the device sustains into a table of
    n_bins doubles at random positions (torch index_add_, one atomic per
    index): the ceiling of a tally scored with HBM atomics."""
    import torch

    g = torch.Generator(device="cuda").manual_seed(7)
    idx = torch.randint(0, n_bins, (n_ops,), device="cuda", generator=g)
    val = torch.ones(n_ops, dtype=torch.float64, device="cuda")
    tab = torch.zeros(n_bins, dtype=torch.float64, device="cuda")
    tab.index_add_(0, idx, val)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(3):
        t0 = time.perf_counter()
        tab.index_add_(0, idx, val)
        torch.cuda.synchronize()
        best = max(best, n_ops / (time.perf_counter() - t0))
    assert float(tab.sum().item()) == 4.0 * n_ops
    del idx, val, tab
    return best


def batched_section(m, w):
    """256 uneven lattices (n x n, n ~ U{4..32}, G ~ U{1..7}, 1e4..1e6
    histories each): the batched solve in both forms (each tuned on its
    first call) against 256 separate runs of the same problems and seeds."""
    import torch

    probs, nh = w.cfg4_batch()
    seeds = [2000 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    log(f"batched: {len(hs)} problems created")
    try:
        res = {"problems": len(probs), "histories": int(sum(nh))}
        outs = {}
        for alg in ("event", "history"):
            m.mcdc_run_batched(hs, nh, seeds, algorithm=alg)      # tunes and caches the launch shape
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs[alg] = m.mcdc_run_batched(hs, nh, seeds, algorithm=alg)
            torch.cuda.synchronize()
            t_b = time.perf_counter() - t0
            res[f"batched_{alg}_s"] = t_b
            res[f"batched_{alg}_histories_per_s"] = sum(nh) / t_b
            log(f"batched {alg} form: {t_b:.3f} s")
        m.mcdc_run_batched(hs, nh, seeds, algorithm="auto")      # times both forms, caches the faster
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.mcdc_run_batched(hs, nh, seeds, algorithm="auto")
        torch.cuda.synchronize()
        res["batched_auto_s"] = time.perf_counter() - t0
        log(f"batched auto form: {res['batched_auto_s']:.3f} s")
        for alg in ("event", "history"):
            m.mcdc_run(hs[0], nh[0], seeds[0], algorithm=alg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            seq = [m.mcdc_run(h, n, s, algorithm=alg) for h, n, s in zip(hs, nh, seeds)]
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
            log(f"batched: {len(hs)} separate {alg} runs {t_s:.3f} s")
            res[f"sequential_{alg}_s"] = t_s
            res[f"speedup_batched_{alg}_vs_sequential_{alg}"] = t_s / res[f"batched_{alg}_s"]
            res[f"counts_match_sequential_{alg}"] = all(
                (a["events"] == b["events"]).all() and (a["terms"] == b["terms"]).all()
                for a, b in zip(outs[alg], seq))
            del seq
        return res
    finally:
        for h in hs:
            h.close()


def fission_section(m, w, n, steps):
    """Supercritical pulse with prompt fission (c = 1.1, one group, 42-mfp
    slab, 20 mean free times): histories/s in both forms and the population
    growth at t = 20 from the time-crossing tally (e^2 = 7.39)."""
    import numpy as np
    import torch

    prob = w.azurv1_supercritical()
    h = m.mcdc_problem_create(prob)
    res = {"workload": "supercritical pulse: 1 group, Sigma_t = v = 1, c = 0.5 + 2.4 x 0.25 = 1.1, "
                       "42-mfp slab, 42 x-bins x 20 time bins on [0, 20] plus the time-crossing tally, "
                       f"{n:.0e} histories", "histories": n}
    try:
        for alg in ("event", "history"):
            out = m.mcdc_run(h, n, 80, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                out = m.mcdc_run(h, n, 81 + s, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[f"{alg}_histories_per_s"] = n / dt
            res[f"{alg}_events_per_s"] = float(sum(out["events"])) / dt
            log(f"fission {alg} form: {dt * 1e3:.1f} ms per run")
        res["events_per_history"] = float(sum(out["events"])) / n
        res["fission_neutrons_per_history"] = out["fission"] / n
        tc = out["tc_mean"].cpu().numpy()[:, 0, 0, 0, :]
        res["population_at_t20"] = float(tc[-1].sum())
        res["population_exact"] = float(np.exp(2.0))
    finally:
        h.close()
    return res


def population_control_section(m, w, n, steps, cpu=True):
    """The pulsed slab with population control at every census edge
    (splitting-roulette, and combing, back to n particles; event form):
    histories/s, the control kernels' share, and the figure of merit
    1/(R^2 T) of the spatially integrated flux in the last time bin against
    the analog run (the population otherwise decays by e^-2 over the 100
    steps)."""
    import numpy as np
    import torch

    prob = w.cfg2_slab_pulse()
    h = m.mcdc_problem_create(prob)
    res = {"workload": "40-mfp slab, c = 0.9, plane pulse at x = 20, 50 x-bins x 100 time bins on [0, 20], "
                       f"{n:.0e} histories, population held at {n:.0e} at each of the 99 inner census edges",
           "histories": n}
    try:
        for tag, kw in (("analog", {}), ("controlled", {"pc_target": n}),
                        ("combed", {"pc_target": n, "pc_method": "comb"})):
            out = m.mcdc_run(h, n, 90, outputs=("mean", "var"), **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                out = m.mcdc_run(h, n, 91 + s, outputs=("mean", "var"), **kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            last = out["mean"].cpu().numpy()[-1].sum()
            var = out["var"].cpu().numpy()[-1].sum()
            rel2 = var / (last * last)
            res[f"{tag}_histories_per_s"] = n / dt
            res[f"{tag}_ms"] = dt * 1e3
            res[f"{tag}_events_per_history"] = float(sum(out["events"])) / n
            res[f"{tag}_last_bin_rel_err"] = float(np.sqrt(rel2))
            res[f"{tag}_last_bin_fom"] = float(1.0 / (rel2 * dt))
            if tag != "analog":
                res[f"{tag}_splits_per_history"] = out["splits"] / n
                res[f"{tag}_rouletted_per_history"] = float(out["terms"][4]) / n
            log(f"population control {tag}: {dt * 1e3:.1f} ms per run")
        res["last_bin_fom_gain"] = res["controlled_last_bin_fom"] / res["analog_last_bin_fom"]
        res["combed_last_bin_fom_gain"] = res["combed_last_bin_fom"] / res["analog_last_bin_fom"]
        # the controlled batches share the weight w_t of every edge, so the
        # batch variance is not that of independent batches: the relative
        # error of one run from the spread of independent replicas instead
        reps = 16
        for tag, kw in (("analog", {}), ("controlled", {"pc_target": n}),
                        ("combed", {"pc_target": n, "pc_method": "comb"})):
            xs = []
            t0 = time.perf_counter()
            for r in range(reps):
                out = m.mcdc_run(h, n, 300 + r, outputs=("mean",), **kw)
                xs.append(float(out["mean"][-1].sum().item()))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            xs = np.array(xs)
            rel = float(xs.std(ddof=1) / xs.mean())
            res[f"{tag}_last_bin_rel_err_replicas"] = rel
            res[f"{tag}_last_bin_fom_replicas"] = float(1.0 / (rel * rel * dt))
        res["replicas"] = reps
        res["last_bin_fom_gain_replicas"] = res["controlled_last_bin_fom_replicas"] / res["analog_last_bin_fom_replicas"]
        res["combed_last_bin_fom_gain_replicas"] = (res["combed_last_bin_fom_replicas"]
                                                    / res["analog_last_bin_fom_replicas"])
        prof = np.zeros((len(m._binding.PROF_CLASSES), 4))
        m.mcdc_run(h, n, 99, outputs=("mean",), pc_target=n, profile=prof, profile_classes=["events", "control"])
        torch.cuda.synchronize()
        ev, ct = m._binding.PROF_CLASSES.index("events"), m._binding.PROF_CLASSES.index("control")
        res["step_kernel_ms"] = float(prof[ev, 0])
        # the three control kernels of every edge (sum, count, apply), each
        # launch bracketed by HIP events: algorithmic bytes (clock words,
        # weights, streams read; whole states read and every copy written)
        # over their device time, against the HBM peak
        res["control_kernels_ms"] = float(prof[ct, 0])
        res["control_launches"] = int(prof[ct, 1])
        res["control_algorithmic_bytes"] = float(prof[ct, 3])
        ach = float(prof[ct, 3] / (prof[ct, 0] * 1e-3) / 1e9) if prof[ct, 0] else None
        res["control_roofline"] = {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                                   "frac": ach / 8000.0 if ach else None}
    finally:
        h.close()
    if cpu:
        # the oracle's census-synchronous run on a bounded sample, one core
        import oracle
        ns = 1_000_000
        oracle.run_pc(prob, 2000, 1, 2000)
        t0 = time.perf_counter()
        oracle.run_pc(prob, ns, 92, ns)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": ns / dt, "unit": "histories/s", "cores": 1, "kind": "oracle",
                               "sample": f"{ns} histories of the same workload with the population held at {ns}"}
        log(f"population control oracle: {dt:.1f} s for {ns} histories")
    return res


def pins_section(m, w, n, steps):
    """Cylindrical-pin geometry: the 17 x 17 lattice of the lattice workload
    with a 0.54-radius fuel pin in every 1.26 cell (7 groups, 17 x 17 x 10 x
    20 bins), both forms; and k-eigenvalue cycles of a reflected pin cell
    with a cylindrical pin (50 inactive + 100 active cycles of 1e5)."""
    import torch

    prob = w.pin_lattice(n=17, n_groups=7, gen_seed=3, height=50.0, n_z_bins=10, n_time_bins=20, t_end=20.0,
                         n_batches=32)
    h = m.mcdc_problem_create(prob)
    res = {"workload": f"17 x 17 pin lattice (pitch 1.26, pin radius 0.54, 7 groups), {n:.0e} histories"}
    try:
        for alg in ("event", "history"):
            out = m.mcdc_run(h, n, 70, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                out = m.mcdc_run(h, n, 71 + s, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[f"{alg}_histories_per_s"] = n / dt
            res[f"{alg}_ms"] = dt * 1e3
            log(f"pins: lattice {alg} form {dt * 1e3:.2f} ms")
        res["events_per_history"] = float(sum(out["events"])) / n
    finally:
        h.close()
    h = m.mcdc_problem_create(w.pin_cell_eigen_cylinder())
    try:
        m.mcdc_run_eigenvalue(h, 100000, 2, 2, 90)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = m.mcdc_run_eigenvalue(h, 100000, 50, 100, 91)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        h.close()
    res["eigen_cylinder_pin_cell"] = {"seconds": dt, "histories_per_s": 1.5e7 / dt, "k_mean": out["k_mean"],
                                      "k_std": out["k_std"]}
    log(f"pins: eigenvalue pin cell {dt:.3f} s, k = {out['k_mean']:.5f} +- {out['k_std']:.5f}")
    return res


def quadrics_section(m, w, n, steps):
    """General quadric surfaces: a 17 x 17 x 10 lattice of 1.26 cubic cells,
    a 0.5-radius spherical fuel kernel in each (7 groups, one tally bin per
    cell, 20 time bins), both forms; and the k-eigenvalue cycles of the
    reflected pin cell with its fuel cylinder written as a general quadric
    (50 inactive + 100 active cycles of 1e5), beside the pin form."""
    import numpy as np
    import torch

    prob = w.sphere_lattice(n=17, n_layers=10, n_groups=7, gen_seed=3, n_time_bins=20, t_end=20.0, n_batches=32)
    h = m.mcdc_problem_create(prob)
    res = {"workload": f"17 x 17 x 10 sphere lattice (pitch 1.26, radius 0.5, 7 groups), {n:.0e} histories"}
    try:
        for alg in ("event", "history"):
            out = m.mcdc_run(h, n, 80, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                out = m.mcdc_run(h, n, 81 + s, algorithm=alg, outputs=("mean",))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[f"{alg}_histories_per_s"] = n / dt
            res[f"{alg}_ms"] = dt * 1e3
            log(f"quadrics: sphere lattice {alg} form {dt * 1e3:.2f} ms")
        res["events_per_history"] = float(sum(out["events"])) / n
    finally:
        h.close()
    cell = w.pin_cell_eigen_cylinder()
    cell["pins"] = None
    c, r = 0.63, 0.54
    cell["quadrics"] = {"coef": np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0, -2.0 * c, -2.0 * c, 0.0,
                                          2.0 * c * c - r * r]).reshape(1, 1, 1, 10),
                        "material": np.zeros((1, 1, 1), dtype=np.int32)}
    h = m.mcdc_problem_create(cell)
    try:
        m.mcdc_run_eigenvalue(h, 100000, 2, 2, 90)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = m.mcdc_run_eigenvalue(h, 100000, 50, 100, 91)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        h.close()
    res["eigen_quadric_pin_cell"] = {"seconds": dt, "histories_per_s": 1.5e7 / dt, "k_mean": out["k_mean"],
                                     "k_std": out["k_std"]}
    log(f"quadrics: eigenvalue pin cell (cylinder as a quadric) {dt:.3f} s, "
        f"k = {out['k_mean']:.5f} +- {out['k_std']:.5f}")
    return res


def eigen_section(m, w, n_per_cycle, n_inactive, n_active):
    """k-eigenvalue power iteration on the box pin cell (7 groups, fuel in
    moderator, reflected), with the cycle counts of Section 3's pin-cell
    test by default (50 inactive + 100 active cycles of 1e5)."""
    import torch

    prob = w.pin_cell_eigen()
    h = m.mcdc_problem_create(prob)
    try:
        m.mcdc_run_eigenvalue(h, n_per_cycle, 2, 2, 90)     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = m.mcdc_run_eigenvalue(h, n_per_cycle, n_inactive, n_active, 91)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        h.close()
    n = n_per_cycle * (n_inactive + n_active)
    log(f"eigenvalue: {dt:.3f} s for {n:.2e} histories, k = {out['k_mean']:.5f} +- {out['k_std']:.5f}")
    return {"workload": f"box pin cell (7 groups, fuel square in moderator, reflective), {n_per_cycle:.0e} "
                        f"per cycle, {n_inactive} inactive + {n_active} active cycles",
            "seconds": dt, "histories_per_s": n / dt, "events_per_s": float(sum(out["events"])) / dt,
            "k_mean": out["k_mean"], "k_std": out["k_std"]}


def pooled(runs):
    """Independent runs of one estimator with equal history counts pooled
    into one estimate: the mean of the means, the variance of that mean
    (sum of the runs' variances over their number squared), the summed
    tracking time, and FOM = 1 / (R^2 T); plus each run's own FOM."""
    k = len(runs)
    mean = sum(r["mean"] for r in runs) / k
    var = sum(r["sigma"] ** 2 for r in runs) / (k * k)
    T = sum(r["T_s"] for r in runs)
    R = math.sqrt(var) / mean if mean > 0 else math.inf
    return {"runs": k, "mean": mean, "sigma": math.sqrt(var), "R": R, "T_s": T,
            "fom": 1.0 / (R * R * T) if mean > 0 else 0.0,
            "fom_per_run": [r["fom"] for r in runs], "splits": sum(r.get("splits", 0) for r in runs)}


def fom_gain(num, den):
    """Ratio of pooled FOMs with a 95 % interval from the spread of the
    runs' own FOMs (log scale, t quantile for the smaller replica count)."""
    g = num["fom"] / den["fom"] if den["fom"] > 0 else None
    if g is None or num["runs"] < 2 or den["runs"] < 2:
        return {"gain": g, "ci95": None}

    def se_log(x):
        v = [math.log(f) for f in x["fom_per_run"]]
        mu = sum(v) / len(v)
        return math.sqrt(sum((a - mu) ** 2 for a in v) / (len(v) - 1) / len(v))

    tq = {1: 12.71, 2: 4.30, 3: 3.18, 4: 2.78, 5: 2.57, 6: 2.45, 7: 2.36, 8: 2.31, 9: 2.26}
    t = tq.get(min(num["runs"], den["runs"]) - 1, 2.0)
    h = t * math.hypot(se_log(num), se_log(den))
    return {"gain": g, "ci95": [g * math.exp(-h), g * math.exp(h)]}


def fom_section(w, pilots, n_analog_run, analog_runs, n_ww, ww_runs, steps):
    """Dog-leg duct, detector behind the second bend (figure of merit
    1/(R^2 T), T the tracking time of the runs): analog Monte Carlo as the
    reference, run as independent replicas until its relative error is
    about 0.05; learned weight windows (forward and adjoint analog pilots,
    network fit on FP32 matrix cores, BF16 inference) built from pilots of
    each size in `pilots`, each judged over independent windowed replicas;
    windows taken straight from the raw adjoint pilot tally (no network);
    and implicit capture.  The pilots take seeds 1000 and 1001, the judged
    runs seeds of their own.  Reported per pilot size: the pooled FOM, the
    FOM with the pilot and training time added to T, the gain over analog
    with its 95 % interval, and the distance of the means in sigma."""
    from paper_2305_07636_amd import learned_ww as lw

    p = w.cfg5_dogleg()
    a_runs = []
    for r in range(analog_runs):
        a_runs.append(lw.figure_of_merit(p, n_analog_run, 5200 + r))
    a = pooled(a_runs)
    log(f"fom: analog {analog_runs} x {n_analog_run:.0e}: mean {a['mean']:.4g} R {a['R']:.4f} "
        f"T {a['T_s']:.2f} s FOM {a['fom']:.3g}")

    def diff(x, y):
        s_ = math.hypot(x["sigma"], y["sigma"])
        return abs(x["mean"] - y["mean"]) / s_ if s_ > 0 else None

    res = {
        "workload": "dog-leg duct 30x10x10, 2 groups, 40x10x10 window mesh, detector box "
                    "[29,30]x[7,9]x[4,6]; history form",
        "analog": dict(a, histories=n_analog_run * analog_runs),
    }
    judged = set()
    for n_pilot in pilots:
        t0 = time.perf_counter()
        table, info = lw.learned_windows(p, n_pilot=n_pilot, steps=steps, seed=1000)
        t_build = time.perf_counter() - t0
        seeds = [5100 + 10 * r + len(res) for r in range(ww_runs)]
        assert not set(seeds) & set(info["pilot_seeds"]) and not set(seeds) & judged
        judged |= set(seeds)
        b = pooled([lw.figure_of_merit(p, n_ww, sd, table=table) for sd in seeds])
        c_seeds = [6100 + 10 * r + len(res) for r in range(2)]
        c = pooled([lw.figure_of_merit(p, n_ww, sd, table=info["raw_table"]) for sd in c_seeds])
        overhead = info["pilot_s"] + info["train_s"]
        fom_incl = 1.0 / (b["R"] ** 2 * (b["T_s"] + overhead)) if b["mean"] > 0 else 0.0
        tag = f"pilot_{n_pilot:.0e}".replace("+", "")
        res[tag] = {
            "pilot_histories": n_pilot, "train_steps": steps, "window_build_s": t_build,
            "pilot_s": info["pilot_s"], "train_s": info["train_s"],
            "loss": [info["loss_first"], info["loss_last"]], "source_resolved": info["source_resolved"],
            "learned": dict(b, histories=n_ww * ww_runs),
            "fom_gain_learned_vs_analog": fom_gain(b, a),
            "fom_incl_pilot_and_training": fom_incl,
            "fom_gain_incl_pilot_and_training": fom_incl / a["fom"] if a["fom"] > 0 else None,
            "mean_diff_sigma_learned_vs_analog": diff(a, b),
            "raw_tally_windows": dict(c, histories=n_ww * 2),
            "fom_gain_raw_vs_analog": c["fom"] / a["fom"] if a["fom"] > 0 else None,
            "fom_gain_learned_vs_raw": b["fom"] / c["fom"] if c["fom"] > 0 else None,
            "mean_diff_sigma_raw_vs_analog": diff(a, c),
        }
        log(f"fom: pilots {n_pilot:.0e}: learned R {b['R']:.4f} T {b['T_s']:.2f} s gain "
            f"{res[tag]['fom_gain_learned_vs_analog']}, incl. pilot+training "
            f"{res[tag]['fom_gain_incl_pilot_and_training']}, mean diff {diff(a, b)} sigma")
    # implicit capture (Section 3 runs the time-dependent duct with it),
    # roulette below weight 0.25 to weight 1
    pic = dict(p, implicit_capture={"w_min": 0.25, "w_survive": 1.0})
    d = pooled([lw.figure_of_merit(pic, n_ww, 5400)])
    res["implicit_capture"] = dict(d, histories=n_ww)
    res["fom_gain_implicit_vs_analog"] = d["fom"] / a["fom"] if a["fom"] > 0 else None
    res["mean_diff_sigma_implicit_vs_analog"] = diff(a, d)
    log(f"fom: implicit capture {d['fom']:.3g}")
    return res


def timed_runs(m, p, N, seed, steps, warmup, alg, counters_file=None, label="slab", bound="alu", n_bins=0):
    """Untimed warm-up runs and one profiled run (HIP events around every
    launch: it names the dominant kernel class), then `steps` timed runs of
    N histories.  In the timed region HIP events bracket only the dominant
    class's launches, on the stream the library launches on; timed run s
    brackets the census steps k = s mod steps, so over the timed region
    every census step is timed once.  Returns histories/s (wall clock over
    the timed runs), the roofline of the dominant kernel and the per-class
    breakdown of the profiled run."""
    import numpy as np
    import torch

    outs = ("mean", "var")
    names = m._binding.PROF_CLASSES

    def run(a, s, **kw):
        return m.mcdc_run(p, N, seed + s, algorithm=a, outputs=outs, **kw)

    for s in range(warmup):
        run(alg, s)
    brk = np.zeros((len(names), 4))
    run(alg, 0, profile=brk)
    cls = int(np.argmax(brk[:, 0]))
    torch.cuda.synchronize()
    prof = np.zeros((len(names), 4))
    t0 = time.perf_counter()
    for s in range(steps):
        last = run(alg, s, profile=prof, profile_classes=[names[cls]], profile_every=steps, profile_phase=s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"{label}: {steps} timed runs of {N:.0e} histories, {elapsed / steps * 1e3:.2f} ms per run")
    ms, launches, items, nbytes = prof[cls]
    if alg == "event":
        # the step kernel takes a chunk's census steps in one launch; every
        # event of the run happens in it
        t_launch = ms / launches * 1e-3
        per_run = brk[cls, 1]
        ev_launch = float(sum(last["events"])) / per_run
        hbm = nbytes / launches / t_launch / 1e9
        cn = measured_counters(counters_file, N) if (counters_file and names[cls] == "events") else None
        traffic = cn["hbm_bytes_per_launch"] if cn else None
        common = {"kernel": "k_event (a chunk's census steps: every particle to death or the last edge)"
                            if names[cls] == "events" else f"k_{names[cls]}",
                  "launches": int(launches), "launches_per_run": int(per_run), "avg_launch_ms": t_launch * 1e3,
                  "events_per_launch": ev_launch,
                  "algorithmic_bytes_per_launch": nbytes / launches, "particles_per_launch": items / launches,
                  "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS},
                  "timed_launches": f"timed run s brackets the launches j = s mod {steps} of the step kernel "
                                    f"with HIP events on the library's stream (each launch once)",
                  "counters_source": os.path.relpath(counters_file, ROOT) if cn else None}
        if bound == "alu":
            # VALU issue: the compiled kernel's VALU instructions per event
            # (SQ_INSTS_VALU over the events of the profiled launches, wave64
            # instructions of 64 lane slots each) times the events of a launch
            per_ev = cn["valu_insts_per_event"] if cn else None
            ach = per_ev * ev_launch * 64 / t_launch / 1e12 if per_ev else None
            roofline = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                        "unit": "TOP/s (VALU lane-operation issue slots)",
                        "frac": ach / VALU_PEAK_TOPS if ach else None, "traffic": traffic,
                        "valu_insts_per_event": per_ev}
        else:
            # FP64 atomics to the HBM tally: the atomics of a launch (its
            # WRITE_SIZE bytes in 32-byte atomic requests) over the device's
            # atomic ceiling measured here
            ceil = atomic_ceiling(n_bins)
            n_at = cn["atomics_per_launch"] if cn else None
            ach = n_at / t_launch / 1e9 if n_at else None
            roofline = {"bound": "atomics", "achieved": ach, "peak": ceil / 1e9,
                        "unit": "G FP64 atomics/s (peak: measured ceiling, torch index_add_ into the "
                                "same number of bins)",
                        "frac": ach / (ceil / 1e9) if ach else None, "traffic": traffic,
                        "atomics_per_launch": n_at}
        roofline.update(common)
    else:
        # history form: state in registers; bounded by FP64 vector ALU and
        # divergence, reported as events per second
        ev = float(sum(last["events"]))
        roofline = {"bound": "alu", "achieved": ev * steps / (ms * 1e-3) / 1e9,
                    "peak": None, "unit": "Gevents/s", "frac": None, "traffic": None,
                    "kernel": "k_history", "launches": int(launches), "avg_launch_ms": ms / launches}
    per_class = {names[c]: {"ms": brk[c, 0], "launches": brk[c, 1], "particles": brk[c, 2],
                            "bytes": brk[c, 3]}
                 for c in range(len(names)) if brk[c, 1] > 0}
    return {"value": N * steps / elapsed, "elapsed": elapsed, "roofline": roofline, "per_class": per_class,
            "last": last}


def sort_section(m, w, n_lattice, steps):
    """The event form's queue sort (two-kernel step, queues reordered by
    event, material, group and cell every c-th census step) against the
    unsorted two-kernel step and the default one-kernel step: the 1e8
    lattice and the 256-problem batch with each step form forced."""
    import torch

    forms = [("one_kernel", {"sort_cadence": -1}), ("two_kernel", {"two_kernel_step": True, "sort_cadence": -1})] + \
        [(f"sorted_every_{c}", {"sort_cadence": c}) for c in (1, 2, 4, 8)]
    res = {"lattice_histories": n_lattice}
    h = m.mcdc_problem_create(w.cfg3_lattice())
    try:
        for tag, kw in forms:
            m.mcdc_run(h, n_lattice, 3, outputs=("mean",), **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                m.mcdc_run(h, n_lattice, 3 + s, outputs=("mean",), **kw)
            torch.cuda.synchronize()
            res[f"lattice_{tag}_ms"] = (time.perf_counter() - t0) / steps * 1e3
            log(f"sort: lattice {tag} {res[f'lattice_{tag}_ms']:.2f} ms")
    finally:
        h.close()
    probs, nh = w.cfg4_batch()
    seeds = [2000 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        for tag, kw in forms:
            for L in (8192, 32768):
                m.mcdc_run_batched(hs, nh, seeds, seg_len=L, **kw)      # tail switch tuned and cached
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m.mcdc_run_batched(hs, nh, seeds, seg_len=L, **kw)
                torch.cuda.synchronize()
                res[f"batched_{tag}_seg{L}_s"] = time.perf_counter() - t0
            log(f"sort: batched {tag} {res[f'batched_{tag}_seg8192_s']:.3f} / {res[f'batched_{tag}_seg32768_s']:.3f} s")
    finally:
        for x in hs:
            x.close()
    return res


def rods_section(m, w, n, steps):
    """A control-rod transient on the lattice workload: the rod bank's tip
    (a moving plane normal to z) descends from z = 50 to z = 10 over the
    first 10 of the 20 time units in every third lattice cell; both forms,
    against the same lattice without rods."""
    import torch

    res = {"workload": "17x17 lattice (7 groups, 17x17x10x20 tally) with a rod bank in every third cell whose tip "
                       f"falls from z=50 to z=10 over t in [0,10]; {n:.0e} histories"}
    for tag, prob in (("rodded", w.rod_lattice()), ("unrodded", w.cfg3_lattice())):
        h = m.mcdc_problem_create(prob)
        try:
            for alg in ("event", "history"):
                out = m.mcdc_run(h, n, 40, algorithm=alg, outputs=("mean",))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for s in range(steps):
                    out = m.mcdc_run(h, n, 41 + s, algorithm=alg, outputs=("mean",))
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / steps
                res[f"{tag}_{alg}_histories_per_s"] = n / dt
                res[f"{tag}_{alg}_ms"] = dt * 1e3
            res[f"{tag}_events_per_history"] = [float(x) / n for x in out["events"]]
            res[f"{tag}_absorbed_fraction"] = float(out["terms"][0]) / n
        finally:
            h.close()
        log(f"rods: {tag} event {res[f'{tag}_event_ms']:.2f} ms, history {res[f'{tag}_history_ms']:.2f} ms")
    return res


def block_section(m, w, n_slab, n_lattice, steps):
    """The event form's census-step kernels at workgroup sizes 256, 512
    and 1024 on the pulsed slab and the lattice."""
    import torch

    res = {}
    cases = [("slab", w.cfg2_slab_pulse(), n_slab, {}), ("slab_staged", w.cfg2_slab_pulse(), n_slab, {"staged": True}),
             ("lattice", w.cfg3_lattice(), n_lattice, {})]
    for tag, prob, n, kw in cases:
        h = m.mcdc_problem_create(prob)
        try:
            for bs in (256, 512, 1024):
                m.mcdc_run(h, n, 2, outputs=("mean",), block_size=bs, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for s in range(steps):
                    m.mcdc_run(h, n, 2 + s, outputs=("mean",), block_size=bs, **kw)
                torch.cuda.synchronize()
                res[f"{tag}_block{bs}_ms"] = (time.perf_counter() - t0) / steps * 1e3
            log(f"block: {tag} " + " ".join(f"{bs}: {res[f'{tag}_block{bs}_ms']:.2f}" for bs in (256, 512, 1024)))
        finally:
            h.close()
    return res


def lattice_section(m, w, n, steps, warmup):
    """The 17 x 17 lattice (2 materials, 7 groups, reflective x-y, vacuum z,
    17 x 17 x 10 x 7 x 20 = 404 600 tally bins, pulse at t = 0) at 1e8
    histories: the event form timed with the roofline of its census-step
    kernel (whose per-step tally slice of 20 230 bins does not fit the LDS,
    so it scores with HBM atomics), and the history form."""
    import torch

    prob = w.cfg3_lattice()
    h = m.mcdc_problem_create(prob)
    res = {"workload": "17x17 lattice of 1.26 cells x 50 high, 2 materials, 7 groups, reflective x/y, vacuum z, "
                       f"uniform pulse at t=0; tally 17x17x10 x 7 groups x 20 time bins on [0,20]; {n:.0e} "
                       "histories, FP64",
           "histories": n}
    try:
        ev = timed_runs(m, h, n, 3, steps, warmup, "event", LATTICE_COUNTERS_FILE, label="lattice event",
                        bound="atomics", n_bins=17 * 17 * 10 * 7 * 20 * 32)
        res["event_histories_per_s"] = ev["value"]
        res["event_ms"] = ev["elapsed"] / steps * 1e3
        res["events_per_history"] = [float(x) / n for x in ev["last"]["events"]]
        res["roofline"] = ev["roofline"]
        res["kernels_per_run"] = ev["per_class"]
        m.mcdc_run(h, n, 3, algorithm="history", outputs=("mean", "var"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            m.mcdc_run(h, n, 3 + s, algorithm="history", outputs=("mean", "var"))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res["history_histories_per_s"] = n / dt
        res["history_ms"] = dt * 1e3
        log(f"lattice history form: {dt * 1e3:.2f} ms per run")
    finally:
        h.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--algorithm", default="event", choices=["event", "history"])
    ap.add_argument("--histories", type=float, default=1e7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-history-form", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fom", action="store_true")
    ap.add_argument("--no-time-crossing", action="store_true")
    ap.add_argument("--no-fission", action="store_true")
    ap.add_argument("--no-eigen", action="store_true")
    ap.add_argument("--no-pins", action="store_true")
    ap.add_argument("--no-quadrics", action="store_true")
    ap.add_argument("--no-pc", action="store_true")
    ap.add_argument("--no-lattice", action="store_true")
    ap.add_argument("--no-sort", action="store_true")
    ap.add_argument("--no-rods", action="store_true")
    ap.add_argument("--no-block", action="store_true")
    ap.add_argument("--lattice-histories", type=float, default=1e8)
    ap.add_argument("--eigen-per-cycle", type=float, default=1e5)
    ap.add_argument("--fission-histories", type=float, default=1e6)
    ap.add_argument("--fom-pilots", default="1e7,1e8", help="pilot sizes of the learned windows")
    ap.add_argument("--fom-analog", type=float, default=4e9, help="histories per analog replica")
    ap.add_argument("--fom-analog-runs", type=int, default=10)
    ap.add_argument("--fom-ww", type=float, default=1e9, help="histories per windowed replica")
    ap.add_argument("--fom-ww-runs", type=int, default=8)
    ap.add_argument("--fom-steps", type=int, default=3000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path (histories would shard by batch with one all-reduce of the "
              "tallies at the end); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    N = int(args.histories)
    seed = 2
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(N, seed)    # before the GPU is touched (spawned workers)
        log(f"cpu baseline: {cpu['value']:.3g} histories/s on {cpu['cores']} processes")

    import numpy as np
    import torch

    import paper_2305_07636_amd as m
    import workloads as w

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    prob = w.cfg2_slab_pulse()
    p = m.mcdc_problem_create(prob)
    outs = ("mean", "var")

    def step(alg, s, **kw):
        return m.mcdc_run(p, N, seed + s, algorithm=alg, outputs=outs, **kw)

    log("problem on the GPU")
    head = timed_runs(m, p, N, seed, args.steps, args.warmup, args.algorithm, COUNTERS_FILE)
    value, elapsed, roofline, per_class, last = (head["value"], head["elapsed"], head["roofline"],
                                                 head["per_class"], head["last"])
    extra = {}
    if not args.no_history_form and args.algorithm == "event":
        torch.cuda.synchronize()
        step("history", 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in range(args.steps):
            step("history", s)
        torch.cuda.synchronize()
        extra["history_form_histories_per_s"] = N * args.steps / (time.perf_counter() - t1)
        log("history form timed")
        # the earlier two-kernel census step (advance, then events), for comparison
        m.mcdc_run(p, N, seed, algorithm="event", outputs=outs, two_kernel_step=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in range(args.steps):
            m.mcdc_run(p, N, seed + s, algorithm="event", outputs=outs, two_kernel_step=True)
        torch.cuda.synchronize()
        extra["two_kernel_step_histories_per_s"] = N * args.steps / (time.perf_counter() - t1)
        # the queue form's kernels, each launch bracketed by HIP events:
        # algorithmic bytes over device time per class
        prof2 = np.zeros((len(m._binding.PROF_CLASSES), 4))
        m.mcdc_run(p, N, seed, algorithm="event", outputs=outs, two_kernel_step=True, profile=prof2)
        torch.cuda.synchronize()
        names = m._binding.PROF_CLASSES
        tk = {}
        for cname in ("advance", "events"):
            c = names.index(cname)
            if prof2[c, 1] > 0:
                ach = prof2[c, 3] / (prof2[c, 0] * 1e-3) / 1e9
                tk[cname] = {"ms": float(prof2[c, 0]), "launches": int(prof2[c, 1]),
                             "particles": float(prof2[c, 2]), "bytes": float(prof2[c, 3]),
                             "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS}
        extra["two_kernel_step_kernels"] = tk
        log("two-kernel step timed")
    if not args.no_time_crossing:
        # the same workload with the time-crossing tally (flux at the 100
        # time edges) as well: its cost in both forms, against runs without
        # it timed the same way (no per-launch events)
        prob_tc = w.cfg2_slab_pulse()
        prob_tc["tally"]["time_crossing"] = True
        ptc = m.mcdc_problem_create(prob_tc)
        tc = {}
        for alg in ("event", "history"):
            for tag, h in (("without", p), ("with", ptc)):
                m.mcdc_run(h, N, seed, algorithm=alg, outputs=outs)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for s in range(args.steps):
                    m.mcdc_run(h, N, seed + s, algorithm=alg, outputs=outs)
                torch.cuda.synchronize()
                tc[f"{alg}_{tag}_histories_per_s"] = N * args.steps / (time.perf_counter() - t1)
            tc[f"{alg}_time_ratio"] = tc[f"{alg}_without_histories_per_s"] / tc[f"{alg}_with_histories_per_s"]
        ptc.close()
        extra["time_crossing_tally"] = tc
        log("time-crossing tally timed")
    p.close()
    if not args.no_lattice:
        extra["lattice"] = lattice_section(m, w, int(args.lattice_histories), args.steps, args.warmup)
    if not args.no_rods:
        extra["moving_plane"] = rods_section(m, w, int(args.histories), args.steps)
    if not args.no_block:
        extra["block_size"] = block_section(m, w, int(args.histories), int(args.lattice_histories), min(args.steps, 3))
    if not args.no_sort:
        extra["queue_sort"] = sort_section(m, w, int(args.lattice_histories), min(args.steps, 3))
    if not args.no_fission:
        extra["fission"] = fission_section(m, w, int(args.fission_histories), args.steps)
    if not args.no_eigen:
        extra["eigenvalue"] = eigen_section(m, w, int(args.eigen_per_cycle), 50, 100)
    if not args.no_pins:
        extra["pins"] = pins_section(m, w, int(args.histories), args.steps)
    if not args.no_quadrics:
        extra["quadrics"] = quadrics_section(m, w, int(args.histories), args.steps)
    if not args.no_pc:
        extra["population_control"] = population_control_section(m, w, int(args.histories), args.steps,
                                                                 cpu=not args.no_cpu_baseline)
    if not args.no_batched:
        extra["batched"] = batched_section(m, w)
    if not args.no_fom:
        extra["figure_of_merit"] = fom_section(w, [int(float(x)) for x in args.fom_pilots.split(",")],
                                               int(args.fom_analog), args.fom_analog_runs, int(args.fom_ww),
                                               args.fom_ww_runs, args.fom_steps)

    line = {
        "metric": METRIC, "value": value, "unit": "histories/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "algorithm": args.algorithm, "histories_per_step": N,
                   "events_per_step": [int(x) for x in last["events"]]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_per_step": per_class,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
