"""Hysteresis of the circular confinement at the paper's coefficients.

The circle section's protocol: starting from the stationary vortex at the
smallest radius, the radius is raised in steps of Delta R, each run starting
from the previous radius's final state, and Psi is measured once the state
has settled; the same downwards from the oscillating state at the largest
radius.  Here both ramps run at once, as two shift-register chains of
instances of one context (one instance per radius and ramp, each with its own
Algorithm 2 mask): after every stage instance j of the upward ramp takes the
final state of instance j - 1 (ttsh_reseed, an exact copy on equal grids, or
with --noise plus projected uniform noise), the downward ramp likewise from
j + 1, and the chain heads keep their own state.  After S stages instance j holds the state continued through the
radii before it on its ramp, as the sequential protocol would, with all
instances busy.  Psi is sampled over the second half of every stage; the
report gives, per ramp and radius, its mean and spread at the last stage
(oscillating states have a spread), and the whole record per stage.

The grid spacing (0.04, box 20.48) is that of the Lyapunov runs, coarser than
the paper's, so the transition radii can differ.  All stepping and
measurement run in the library; the statistics are host-side analysis.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def run(radii, stages=None, steps=40_000, every=100, N=512, L=20.48, seed=5, log=None, dt: float = 0.01,
        noise: float = 0.0) -> dict:
    params = dataclasses.replace(W.paper_coefficients(dt=dt))
    nr = len(radii)
    stages = stages or nr
    up = list(range(nr))             # instance of radius j on the upward ramp
    down = list(range(nr, 2 * nr))   # ... on the downward ramp
    n = 2 * nr
    s = T.Solver([N] * n, [L] * n, params, T.TTSH_FP32)
    try:
        s.option(T.TTSH_OPT_GRAPH_STEPS, every)
        for j, R in enumerate(radii):
            for q in (up[j], down[j]):
                s.mask_from_binary(q, W.binary_outside(N, L, [(0.0, 0.0)], [R]))
                s.set_field(q, W.uniform_field(seed + q, N, 0.01, 32))
        s.tune(every)
        t0 = time.time()
        nsamp = (steps // 2) // every
        record = []
        for st in range(stages):
            s.step(steps - nsamp * every)
            psi = np.zeros((nsamp, n))
            for k in range(nsamp):
                s.step(every)
                for q in range(n):
                    psi[k, q] = s.order(q)[0]
            record.append({"mean": psi.mean(axis=0).tolist(), "std": psi.std(axis=0).tolist()})
            if log:
                log(f"stage {st + 1}/{stages}: up Psi {np.round(psi.mean(axis=0)[:nr], 3).tolist()}, "
                    f"down Psi {np.round(psi.mean(axis=0)[nr:], 3).tolist()}")
            if st + 1 < stages:
                dst = up[1:] + down[:-1]
                src = up[:-1] + down[1:]
                # projected uniform noise on every hand-off (none if noise == 0),
                # drawn on the device
                s.reseed(dst, src, noise, seed + 7919 * (st + 1))
        s.sync()
        secs = time.time() - t0
        last = record[-1]
        table = [{"R": R, "up_psi": last["mean"][up[j]], "up_std": last["std"][up[j]],
                  "down_psi": last["mean"][down[j]], "down_std": last["std"][down[j]]}
                 for j, R in enumerate(radii)]
        return {"N": N, "L": L, "dt": dt, "steps_per_stage": steps, "stages": stages, "sample_every": every,
                "handoff_noise": noise,
                "coefficients": "paper preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)",
                "mask": "Algorithm 2 from the binary outside-the-circle field",
                "seconds": secs, "radii": table, "record": record}
    finally:
        s.close()


def main(argv=None):
    """Up and down ramps of the circle radius at the paper's coefficients."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--radii", type=float, nargs="+",
                    default=[5.16, 5.18, 5.20, 5.22, 5.24, 5.26, 5.28, 5.30, 5.32, 5.34, 5.36, 5.38])
    ap.add_argument("--stages", type=int, default=0, help="default: one per radius")
    ap.add_argument("--steps", type=int, default=40_000, help="steps per stage")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--L", type=float, default=20.48)
    ap.add_argument("--noise", type=float, default=0.0,
                    help="amplitude of projected uniform noise added at every hand-off (0: exact copies)")
    ap.add_argument("--report", default="hysteresis_report.json")
    a = ap.parse_args(argv)
    rep = run(a.radii, a.stages or None, a.steps, a.every, a.N, a.L,
              log=lambda m: print(f"[hysteresis] {m}", flush=True), noise=a.noise)
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f)
    print(f"[hysteresis] {2 * len(a.radii)} instances of {a.N}^2, {rep['stages']} stages of {a.steps} steps "
          f"in {rep['seconds']:.1f} s", flush=True)
    for r in rep["radii"]:
        print(f"[hysteresis] R={r['R']:.2f}: up Psi {r['up_psi']:.3f} +- {r['up_std']:.3f}, "
              f"down Psi {r['down_psi']:.3f} +- {r['down_std']:.3f}", flush=True)
    return rep


if __name__ == "__main__":
    main()
