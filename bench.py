#!/usr/bin/env python
"""Throughput of the TTSH time step on one MI355X.

Headline ("value"): the batched radius sweep in FP32 -- 64 instances, radii
8..80 on 128^2, 256^2 and 512^2 grids (box side 3.2 R), all advanced together;
a "step" is one time step of every instance (10,682,368 grid points).  Also
reported: the plain single-instance 512^2 run ("plain"), the FP32-vs-FP64
oracle error at step 1000 of both ("parity"), the roofline figure of the
dominant kernel from HIP-event timings taken in this process, and the FP64 CPU
oracle timed on a bounded sample of the same workload ("cpu_baseline").

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "grid-pt·steps/s batched vs plain at L2 err ≤1e-5 vs FP64; % HBM peak"
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_step_kernels_radius_sweep.json")
STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats_step_kernels_radius_sweep.json")
STEP_SOURCES = ("common.hpp", "fft.hpp", "step.hpp", "step_multi.hpp", "step_multi.hip", "step_sched.hip")


def step_source_hash() -> str:
    """SHA-256 over the sources that define the two step kernels; a traffic
    measurement is only reported while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2304_03306_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def source_revision():
    """Git commit of the tree (with a mark if it has local changes), or None."""
    import subprocess
    try:
        rev = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short", "HEAD"], capture_output=True, text=True,
                             timeout=10).stdout.strip()
        dirty = subprocess.run(["git", "-C", ROOT, "status", "--porcelain", "--untracked-files=no"],
                               capture_output=True, text=True, timeout=10).stdout.strip()
        return (rev + ("+local-changes" if dirty else "")) or None
    except (OSError, subprocess.SubprocessError):
        return None


def _pmc_means(path: str, counter: str) -> dict:
    """Mean counter value per kernel name over the dispatches of a rocprofv3
    counter_collection.csv."""
    import csv
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            a = acc.setdefault(r["Kernel_Name"], [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    return {k: v[0] / v[1] for k, v in acc.items()}


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib) -> dict:
    """HBM bytes per dispatch of the step kernels from FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch), scaled by what the same counters read for a
    device copy of copy_mib MiB (bytes moved per counted byte)."""
    copy_bytes = copy_mib * (1 << 20)
    cf = [v for k, v in _pmc_means(copy_fetch_csv, "FETCH_SIZE").items() if "copyBuffer" in k]
    cw = [v for k, v in _pmc_means(copy_write_csv, "WRITE_SIZE").items() if "copyBuffer" in k]
    fscale = copy_bytes / (cf[0] * 1024.0)
    wscale = copy_bytes / (cw[0] * 1024.0)
    fetch, write = _pmc_means(fetch_csv, "FETCH_SIZE"), _pmc_means(write_csv, "WRITE_SIZE")
    kernels = {}
    for name in fetch:
        if ("row_multi" in name or "col_multi" in name) and name in write:
            kernels[name] = {"fetch_kib": fetch[name], "write_kib": write[name],
                             "bytes": fetch[name] * 1024.0 * fscale + write[name] * 1024.0 * wscale}
    return {"source_sha256": step_source_hash(), "fetch_scale": fscale, "write_scale": wscale,
            "copy_mib": copy_mib, "kernels": kernels}


def kernel_name(pass_: str, block: int, sched: int, state_bytes: int = 8) -> str:
    """The profiler's name of a multi-size step kernel of the FP32 transforms
    (no vorticity damping; column pass in its one-stage form)."""
    if pass_ == "row":
        return f"void ttsh::row_multi<float, false, {block}, {sched}>(ttsh::MultiArgs)"
    S = "float" if state_bytes == 8 else "double"
    return f"void ttsh::col_multi<float, {S}, false, 0, {block}, {sched}>(ttsh::MultiArgs)"


def measured_traffic(name: str):
    """Bytes per launch of the named step kernel from the committed counter
    summary, or None if it is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != step_source_hash():
        return None
    v = t.get("kernels", {}).get(name)
    return v["bytes"] if v else None


def summarize_stats(stats_csv) -> dict:
    """Mean duration per kernel name from a rocprofv3 --stats kernel_stats.csv."""
    import csv
    kernels = {}
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            kernels[r["Name"]] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                                  "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3}
    return {"source_sha256": step_source_hash(), "kernels": kernels}


def recorded_avg_us(name: str):
    """The rocprofv3 mean duration of the named step kernel from the committed
    summary, or None if it is missing or the kernel sources changed since."""
    try:
        with open(STATS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != step_source_hash():
        return None
    v = t.get("kernels", {}).get(name)
    return v["avg_us"] if v else None


def stream_ceiling(torch, T, mib: int = 160, reps: int = 30):
    """Rates of the library's streaming probe for several read:write mixes, on
    arrays totalling about `mib` MiB (the size of one step pass's traffic) and
    on 2 GiB (beyond the 256 MB last-level cache).  GB/s = bytes moved per
    launch / mean launch time; the best workgroup count of a few is kept."""
    out = {}
    for total_mib in (mib, 2048):
        for r, w in ((1, 1), (2, 1), (5, 2), (1, 0)):
            arrays = r + w
            elems = total_mib * (1 << 20) // (16 * arrays)
            buf = torch.zeros((r + max(w, 1)) * elems * 4, dtype=torch.float32, device="cuda")
            best = 0.0
            for blocks in (2048, 8192, 32768):
                us = T.ttsh_stream_bench(r, w, elems, blocks, reps if total_mib <= 256 else 5, buf)
                best = max(best, arrays * elems * 16 / (us * 1e-6) / 1e9)
            out[f"{total_mib}MiB_r{r}w{w}"] = round(best, 1)
            del buf
    torch.cuda.synchronize()
    return out


def kept_modes(N: int) -> int:
    """Stored modes per component that the 1/2 rule keeps: m_x = 0..M,
    m_y = -M..M with m_x^2 + m_y^2 <= M^2 (M = N/4)."""
    M = N // 4
    return sum(2 * int(np.floor(np.sqrt(M * M - mx * mx))) + 1 for mx in range(M + 1))


def pass_bytes(N: int, state_bytes: int = 8, gw: bool = False) -> tuple[int, int]:
    """Algorithmic HBM bytes of one instance for (row pass, column pass);
    FP32 transforms, `state_bytes` per stored complex mode.

    Row pass:    read v_x, v_y, omega in the mixed domain (3 (M+1) N complex),
                 read K (N^2 reals), write the forcing (2 (M+1) N complex) and
                 the row sums (2N reals).
    Column pass: read the forcing, read and write the kept modes of the state
                 (2 components), write the mixed v_x, v_y, omega, read the row
                 sums.
    """
    M = N // 4
    c8, r4 = 8, 4
    nf = 3 if gw else 2
    mixed = (M + 1) * N * c8
    row = 3 * mixed + N * N * r4 + nf * mixed + 2 * N * r4
    col = nf * mixed + 2 * 2 * kept_modes(N) * state_bytes + 3 * mixed + 2 * N * r4
    return row, col


def setup(T, W, wl, params, prec):
    s = T.Solver([i.N for i in wl.instances], [i.L for i in wl.instances], params, prec)
    for q, inst in enumerate(wl.instances):
        s.mask_tanh(q, inst.centers, inst.radii, inst.xi)
        s.set_field(q, W.uniform_field(inst.seed, inst.N, 0.01, 32))
    return s


def reinit(s, W, wl):
    for q, inst in enumerate(wl.instances):
        s.set_field(q, W.uniform_field(inst.seed, inst.N, 0.01, 32))


def golden_rel_l2(s, q, name):
    """rel-L2 of instance q against a stored FP64 oracle state (Parseval on
    the compact spectrum: m_x > 0 columns count twice)."""
    path = os.path.join(GOLDEN, f"ref_{name}_step1000.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)["state"].astype(np.complex128)
    got = s.state(q)
    w = np.ones(ref.shape[-1])
    w[1:] = 2.0
    num = np.sum(w * np.abs(got - ref) ** 2)
    den = np.sum(w * np.abs(ref) ** 2)
    return float(np.sqrt(num / den))


def timed_steps(s, torch, steps):
    torch.cuda.synchronize()
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(wl, budget_s: float):
    """The FP64 oracle (Algorithm 1 as printed) on the host cores: per distinct
    grid size one instance of the workload is stepped for a bounded number of
    steps; the per-point rates are combined with the workload's size mix."""
    from oracle import ttsh as O
    from paper_2304_03306_amd import workloads as W
    p = O.workload_params()
    sizes = sorted({i.N for i in wl.instances})
    per = budget_s / len(sizes)
    sec_per_pt = {}
    sample = []
    for N in sizes:
        inst = next(i for i in wl.instances if i.N == N)
        K = O.mask_tanh(N, inst.L, inst.centers, inst.radii, inst.xi)
        v, w = O.alg1_init(W.uniform_field(inst.seed, N, 0.01, 32), inst.L)
        t0 = time.perf_counter()
        v, w = O.alg1_step(v, w, K, p, inst.L)  # warm-up (plans, caches)
        one = time.perf_counter() - t0
        n = max(2, min(200, int(per / max(one, 1e-4))))
        t0 = time.perf_counter()
        for _ in range(n):
            v, w = O.alg1_step(v, w, K, p, inst.L)
        dt = time.perf_counter() - t0
        sec_per_pt[N] = dt / (n * N * N)
        sample.append(f"{n} steps of one {N}^2 instance")
    t_step = sum(sec_per_pt[i.N] * i.N * i.N for i in wl.instances)
    return {"value": wl.points / t_step, "unit": "grid-pt·steps/s", "cores": os.cpu_count(),
            "kind": "oracle",
            "sample": "FP64 Algorithm-1 oracle (scipy.fft, workers=all cores): " + ", ".join(sample)
                      + "; per-point rates combined with the workload's grid-size mix"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--prof-steps", type=int, default=100, help="steps timed per kernel with HIP events")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--workload", default="sweep", choices=["sweep", "dumbbell"])
    ap.add_argument("--precision", type=int, default=32, choices=[32, 96],
                    help="32: FP32 state; 96: FP64 state (FP32 transforms in both)")
    ap.add_argument("--block", type=int, default=0, help="workgroup size (0 = autotuned)")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON cache of tuner results (default: the package's tuning_cache.json)")
    ap.add_argument("--retune", action="store_true", help="tune even if the cache holds a choice")
    ap.add_argument("--groups", type=int, default=0, choices=[0, 1, 2],
                    help="concurrent instance groups of the step (0 = the tuned choice); 1 gives "
                         "profiles whose step kernels run alone, as the roofline's per-kernel figure")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 10 times (scale for the HBM byte counters)")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming-bandwidth probe")
    ap.add_argument("--summarize-stats", metavar="KERNEL_STATS_CSV",
                    help="write the rocprofv3 mean durations of the step kernels (read back by later runs)")
    ap.add_argument("--summarize-pmc", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV", "COPY_MIB"),
                    help="write the HBM traffic summary of the step kernels from rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.summarize_stats:
        summary = summarize_stats(args.summarize_stats)
        with open(STATS_FILE, "w") as f:
            json.dump(summary, f, indent=1)
        print(json.dumps(summary, indent=1))
        return
    if args.summarize_pmc:
        a = args.summarize_pmc
        summary = summarize_pmc(a[0], a[1], a[2], a[3], int(a[4]))
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(summary, f, indent=1)
        print(json.dumps(summary, indent=1))
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * n * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"[bench] copied {args.copy_calibration} MiB 11 times: {gbs:.0f} GB/s read + write")
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the workloads shard by instance; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_03306_amd import ttsh as T, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    params = W.workload_coefficients()
    wl = W.radius_sweep() if args.workload == "sweep" else W.dumbbells()
    log(f"[bench] workload {wl.name}: {len(wl.instances)} instances, {wl.points} points/step")
    state_bytes = 8 if args.precision == 32 else 16
    s = setup(T, W, wl, params, args.precision)
    # the NaN/Inf guard stays on, as in production runs: the step graphs carry a
    # check of every instance each 50 steps and ttsh_sync checks once more
    from paper_2304_03306_amd import tuning
    cache = args.tuning_cache or tuning.DEFAULT_CACHE
    if args.block:
        s.option(T.TTSH_OPT_BLOCK, args.block)
        cfg = s.get_tuning()
    else:
        cfg, tuned_us, hit = tuning.autotune(s, 20, cache, retune=args.retune)
        log(f"[bench] {'tuning from the cache' if hit else 'autotuned'}: (row, column) workgroup sizes "
            f"{cfg[:2]}, one launch per grid size {cfg[2:4]}, transform schedules {cfg[4:6]}, "
            f"concurrent instance groups {cfg[6] if len(cfg) > 6 else 1}"
            + (f" ({tuned_us:.1f} us/step when tuned)" if tuned_us else ""))
        cfg = s.get_tuning()
    if args.groups:
        s.option(T.TTSH_OPT_GROUPS, args.groups)
        cfg = s.get_tuning()
    block, split, sched, groups = tuple(cfg[0:2]), tuple(cfg[2:4]), tuple(cfg[4:6]), int(cfg[6])

    parity = {}
    if not args.no_parity and args.workload == "sweep":
        s.step(1000)
        s.sync()
        for q, name in ((0, "sweep_R8_128"), (14, "sweep_R24_256"), (62, "sweep_R80_512")):
            parity[name] = golden_rel_l2(s, q, name)
        log(f"[bench] parity at step 1000: {parity}")
        reinit(s, W, wl)

    # warm-up; a call whose length is not a whole number of graph chunks ends
    # with a tail graph of its own length, so one untimed call of that tail
    # captures it before the timed region
    tail = args.steps % 50
    warmup = args.warmup + tail
    s.step(args.warmup)
    if tail:
        s.step(tail)
    s.sync()
    dt = timed_steps(s, torch, args.steps)
    value = wl.points * args.steps / dt
    log(f"[bench] {args.steps} steps in {dt:.3f} s: {value:.4e} pt*steps/s")
    finite = True
    try:
        s.sync()
    except T.TTSHError:
        finite = False

    # per-kernel durations from HIP events on the library's stream: every
    # instance in one launch, launches back to back and alone on the GPU (with
    # two instance groups the step's launches cover half the instances each
    # and overlap, so their own durations say nothing about one kernel; the
    # whole step's rate is in step_hbm)
    row_us, col_us = T.ttsh_pass_times(s.ctx, args.prof_steps)
    counts = {}
    for i in wl.instances:
        counts[i.N] = counts.get(i.N, 0) + 1
    row_b = sum(pass_bytes(N, state_bytes)[0] * n for N, n in counts.items())
    col_b = sum(pass_bytes(N, state_bytes)[1] * n for N, n in counts.items())
    # kernel names as the profiler shows them: one launch per grid size runs row_one / col_one
    kern = [("row_one" if split[0] else "row_multi", row_us, row_b, block[0], sched[0], "row"),
            ("col_one" if split[1] else "col_multi", col_us, col_b, block[1], sched[1], "col")]
    dom = max(kern, key=lambda k: k[1])
    # the recorded counter and duration summaries are of the radius sweep
    recorded = args.workload == "sweep" and not split[kern.index(dom)]
    dom_name = kernel_name(dom[5], dom[3], dom[4], state_bytes) if recorded else None
    traffic = measured_traffic(dom_name) if recorded and args.precision == 32 else None
    achieved = dom[2] / (dom[1] * 1e-6) / 1e9
    rocprof_us = recorded_avg_us(dom_name) if recorded else None
    step_bytes = row_b + col_b
    step_us = row_us + col_us
    log("[bench] kernels: " + ", ".join(f"{k[0]} {k[1]:.1f}us {k[2] / k[1] / 1e3:.0f}GB/s" for k in kern))
    s.close()

    plain = None
    if not args.no_plain:
        pw = W.circle_fp32_512()
        ps = setup(T, W, pw, params, args.precision)
        pcfg, _, _ = tuning.autotune(ps, 20, cache, retune=args.retune)
        pblock = pcfg[:2]
        perr = None
        if not args.no_parity:
            ps.step(1000)
            ps.sync()
            perr = golden_rel_l2(ps, 0, "circle512")
            parity["circle512"] = perr
            reinit(ps, W, pw)
        ps.step(args.warmup)
        psteps = args.steps * 2
        pdt = timed_steps(ps, torch, psteps)
        plain = {"workload": pw.name, "value": pw.points * psteps / pdt, "unit": "grid-pt·steps/s",
                 "steps": psteps, "ms_per_step": 1e3 * pdt / psteps,
                 "config": {"N": 512, "L": 256.0, "R": 60.0, "instances": 1, "block": pblock}}
        log(f"[bench] plain 512^2: {plain['value']:.4e} pt*steps/s, {plain['ms_per_step'] * 1e3:.1f} us/step")
        ps.close()

    stream = None
    if not args.no_stream:
        stream = stream_ceiling(torch, T)
        log(f"[bench] streaming probe (GB/s): {stream}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_budget)
        log(f"[bench] cpu baseline {cpu['value']:.4e} pt*steps/s on {cpu['cores']} cores")

    sizes = sorted(counts)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-pt·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f32 (f64 state)",
        "data": "synthetic",
        "config": {"workload": wl.name, "instances": len(wl.instances),
                   "grids": " + ".join(f"{counts[N]}x{N}^2" for N in sizes),
                   "points_per_step": wl.points, "dt": params.dt, "block": block,
                   "launch_per_grid_size": split, "transform_schedule": sched,
                   "concurrent_groups": groups,
                   "precision": ("FP32 transforms and state" if args.precision == 32 else
                                 "FP32 transforms, FP64 state") + ", FP64 k-space update",
                   "parallelism": "single GPU, instances batched per grid size"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dom_name or dom[0], "block": dom[3], "schedule": dom[4], "avg_us": dom[1],
                     "bytes_per_launch": dom[2],
                     "rocprof_avg_us": rocprof_us,
                     "rocprof_frac": (dom[2] / (rocprof_us * 1e-6) / 1e9 / HBM_PEAK_GBS) if rocprof_us else None},
        "stream_probe_GBps": stream,
        "step_hbm": {"algorithmic_bytes": step_bytes, "kernel_us": step_us,
                     "GBps": step_bytes / (step_us * 1e-6) / 1e9,
                     "frac": step_bytes / (step_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "wall_GBps": step_bytes * args.steps / dt / 1e9,
                     "wall_frac": step_bytes * args.steps / dt / 1e9 / HBM_PEAK_GBS,
                     "concurrent_groups": groups},
        "parity": {"rel_l2_step1000_vs_fp64_oracle": parity, "all_finite": finite},
        "plain": plain,
        "cpu_baseline": cpu,
        "source": source_revision(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
