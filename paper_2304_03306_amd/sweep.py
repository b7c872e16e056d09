"""Batched radius sweep with continuation: the hysteresis scan of the circle
section run for all radii at once.

All 64 instances of the radius sweep (32 radii, each on an upward and a
downward ramp) advance together in one context.  After every stage each
instance is reseeded from its chain predecessor's final state -- the upward
ramp from the next smaller radius, the downward ramp from the next larger one
(ttsh_reseed: mode-index transfer between the grids, plus projected uniform
noise) -- so that after S stages instance j of a ramp has been continued
through the S radii before it, as the sequential protocol would, but with all
instances busy.  The vortex order parameter Psi of every instance and its
vortex count (centres and saddles of the velocity direction inside the
circle, ttsh_vortices) are taken at the end of each stage.

Every step of the computation runs in the library; this module orders the
calls and keeps the record.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def run(stages: int, steps: int, log=None, tune: bool = True, scheme: str = "ifeuler") -> dict:
    import dataclasses
    wl = W.radius_sweep()
    inst = wl.instances
    n = len(inst)
    params = dataclasses.replace(W.workload_coefficients(), scheme=scheme)
    s = T.Solver([i.N for i in inst], [i.L for i in inst], params, T.TTSH_FP32)
    try:
        for q, i in enumerate(inst):
            s.mask_tanh(q, i.centers, i.radii, i.xi)
            s.set_field(q, W.uniform_field(i.seed, i.N, 0.01, 32))
        if tune:
            s.tune(20)
        src = W.sweep_chain(n // 2)
        psi = np.zeros((stages, n))
        centres = np.zeros((stages, n), dtype=np.int64)
        saddles = np.zeros((stages, n), dtype=np.int64)
        seconds = []
        for st in range(stages):
            t0 = time.time()
            s.step(steps)
            s.sync()
            seconds.append(time.time() - t0)
            for q in range(n):
                psi[st, q] = s.order(q, inst[q].centers[0])[0]
                # nodes slower than 1e-3 of the rms speed have no defined direction
                vmin = 1e-3 * np.sqrt(s.norms(q)[0] / inst[q].N ** 2)
                centres[st, q], saddles[st, q] = s.vortices(q, 0.5, vmin)
            if log:
                log(f"stage {st}: {steps} steps in {seconds[-1]:.2f} s; "
                    f"Psi up {np.round(psi[st, 0::2], 2).tolist()}")
            if st + 1 < stages:
                # U[-1e-3, 1e-3] noise per node, drawn on the device (Philox)
                s.reseed(list(range(n)), src, 1e-3, W.stage_seed(st))
        radii = [inst[2 * j].radii[0] for j in range(n // 2)]
        return {"radii": radii, "stages": stages, "steps_per_stage": steps,
                "psi_up": psi[:, 0::2].tolist(), "psi_down": psi[:, 1::2].tolist(),
                "centres_up": centres[:, 0::2].tolist(), "centres_down": centres[:, 1::2].tolist(),
                "saddles_up": saddles[:, 0::2].tolist(), "saddles_down": saddles[:, 1::2].tolist(),
                "seconds_per_stage": seconds,
                "points_per_step": wl.points,
                "throughput": wl.points * steps / float(np.mean(seconds))}
    finally:
        s.close()


def main(argv=None):
    """Hysteresis scan over the radius sweep; writes a JSON report."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--stages", type=int, default=32)
    ap.add_argument("--steps", type=int, default=20_000)
    ap.add_argument("--scheme", default="ifeuler", choices=["ifeuler", "etd1", "imex", "etdrk2", "etdrk4"])
    ap.add_argument("--report", default="sweep_report.json")
    a = ap.parse_args(argv)
    rep = run(a.stages, a.steps, log=lambda m: print(f"[sweep] {m}", flush=True), scheme=a.scheme)
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f, indent=1)
    print(f"[sweep] {a.stages} stages of {a.steps} steps; {rep['throughput']:.4e} pt*steps/s", flush=True)
    return rep


if __name__ == "__main__":
    main()
