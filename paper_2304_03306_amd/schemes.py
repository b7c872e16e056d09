"""Accuracy against cost of the time steppers on the radius sweep.

The 64 sweep instances are advanced from their seeded starts to a common time
T with the paper's integrating-factor Euler step (Algorithm 1) and with the
exponential Runge-Kutta steps of second and fourth order (ETD2RK, ETDRK4) at
several time steps.  The error of each run is the mean over instances of the
relative L2 difference, at T, from a reference run of ETDRK4 with a time step
eight times smaller than the finest one compared; these accuracy runs use
FP64 arithmetic so that rounding stays far below the time-stepping error.  The
cost of each configuration is the wall time of the same run in FP32 (the
production arithmetic), workgroup sizes tuned per scheme.

Every step runs in the library; this module orders the calls and compares
the fields it reads back.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def _solver(inst, params, prec, tune_steps=0):
    s = T.Solver([i.N for i in inst], [i.L for i in inst], params, prec)
    for q, i in enumerate(inst):
        s.mask_tanh(q, i.centers, i.radii, i.xi)
        s.set_field(q, W.uniform_field(i.seed, i.N, 0.01, 32))
    if tune_steps:
        s.tune(tune_steps)
    return s


def _fields(s, n):
    return [s.field(q) for q in range(n)]


def run(T_end: float = 2.0, dts=(0.02, 0.01, 0.005, 0.0025), schemes=("ifeuler", "etdrk2", "etdrk4"),
        log=None) -> dict:
    inst = W.radius_sweep().instances
    n = len(inst)
    base = W.workload_coefficients()
    dt_ref = min(dts) / 8
    ref_p = dataclasses.replace(base, dt=dt_ref, scheme="etdrk4")
    s = _solver(inst, ref_p, T.TTSH_FP64)
    try:
        s.step(int(round(T_end / dt_ref)))
        s.sync()
        ref = _fields(s, n)
    finally:
        s.close()
    norms = [float(np.sqrt(np.sum(r * r))) for r in ref]
    rows = []
    for scheme in schemes:
        for dt in dts:
            steps = int(round(T_end / dt))
            p = dataclasses.replace(base, dt=dt, scheme=scheme)
            s = _solver(inst, p, T.TTSH_FP64)
            try:
                s.step(steps)
                s.sync()
                got = _fields(s, n)
            finally:
                s.close()
            errs = [float(np.sqrt(np.sum((g - r) ** 2))) / nr for g, r, nr in zip(got, ref, norms)]
            finite = all(np.isfinite(e) for e in errs)
            s = _solver(inst, p, T.TTSH_FP32, tune_steps=20)
            try:
                s.step(min(steps, 50))  # warm-up (graph build)
                s.sync()
                t0 = time.perf_counter()
                s.step(steps)
                s.sync()
                secs = time.perf_counter() - t0
            finally:
                s.close()
            row = {"scheme": scheme, "dt": dt, "steps": steps,
                   "mean_rel_l2": float(np.mean(errs)) if finite else float("nan"),
                   "max_rel_l2": float(np.max(errs)) if finite else float("nan"),
                   "fp32_seconds": secs, "fp32_ms_per_step": 1e3 * secs / steps}
            rows.append(row)
            if log:
                log(f"{scheme} dt={dt}: {steps} steps, mean rel-L2 {row['mean_rel_l2']:.3e}, "
                    f"FP32 {row['fp32_ms_per_step']:.3f} ms/step, {secs:.3f} s")
    return {"workload": "radius_sweep (64 instances: 12 x 128^2, 16 x 256^2, 36 x 512^2)",
            "T": T_end, "reference": {"scheme": "etdrk4", "dt": dt_ref, "precision": "FP64"},
            "runs": rows}


def main(argv=None):
    """Error at a common time against FP32 cost, per stepper and time step."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--T", type=float, default=2.0)
    ap.add_argument("--dts", type=float, nargs="+", default=[0.02, 0.01, 0.005, 0.0025])
    ap.add_argument("--schemes", nargs="+", default=["ifeuler", "etdrk2", "etdrk4"],
                    choices=["ifeuler", "etd1", "imex", "etdrk2", "etdrk4"])
    ap.add_argument("--report", default="schemes_report.json")
    a = ap.parse_args(argv)
    rep = run(a.T, tuple(a.dts), tuple(a.schemes), log=lambda m: print(f"[schemes] {m}", flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f, indent=1)
    return rep


if __name__ == "__main__":
    main()
