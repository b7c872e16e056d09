"""Dumbbell confinement with the paper's coefficients: Psi_2 against the
centre-to-centre distance D for several cavity radii R.

The dumbbell section's set-up: two overlapping circles of radius R (near the
size of one vortex, R ~ pi) whose centres are D apart, the mask built by
Algorithm 2 from the binary field that is 1 outside both circles (the logical
AND of the two "outside" fields), the paper's preset (a, b, lambda, gamma_v,
gamma_w) = (0.5, 1.6, 9, 40, 4), random small initial fields.  Every (R, D)
pair, with several seeds, is one instance of a single context.  After a
transient, Psi_2 (vorticity peaks in the disks of radius D/2 about the two
cavity centres, ttsh_order_dumbbell) and the vortex count are sampled at
fixed intervals; the report gives, per (R, D), the mean Psi_2 over samples
and seeds and the distance at which it falls through 1/2.  The grid spacing
is that of the circle driver (0.04), coarser than the paper's.

All time stepping and measurement run in the library; the statistics of the
sampled series are host-side analysis of its output.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def run(radii, ratios, seeds=2, N=512, L=20.48, steps=100_000, transient=60_000, every=500, seed0=11,
        log=None, scheme: str = "ifeuler", dt: float = 0.01) -> dict:
    params = dataclasses.replace(W.paper_coefficients(dt=dt), scheme=scheme)
    cases = [(R, round(f * R, 6), s) for R in radii for f in ratios for s in range(seeds)]
    n = len(cases)
    s = T.Solver([N] * n, [L] * n, params, T.TTSH_FP32)
    try:
        s.option(T.TTSH_OPT_GRAPH_STEPS, every)
        for q, (R, D, k) in enumerate(cases):
            s.mask_from_binary(q, W.binary_outside(N, L, [(-D / 2, 0.0), (D / 2, 0.0)], [R, R]))
            s.set_field(q, W.uniform_field(seed0 + 1000 * k + q, N, 0.01, 32))
        s.tune(every)
        t0 = time.time()
        s.step(transient)
        s.sync()
        nsamp = (steps - transient) // every
        psi2 = np.zeros((nsamp, n))
        centres = np.zeros((nsamp, n), dtype=np.int64)
        for j in range(nsamp):
            s.step(every)
            for q, (R, D, k) in enumerate(cases):
                psi2[j, q] = s.order_dumbbell(q, D)
                sq = s.norms(q)[0]
                centres[j, q] = s.vortices(q, 0.5, 1e-3 * np.sqrt(sq / (N * N)))[0]
            if log and (j + 1) % max(1, nsamp // 5) == 0:
                log(f"sample {j + 1}/{nsamp}: mean Psi_2 {float(np.nanmean(psi2[j])):.3f}")
        s.sync()
        secs = time.time() - t0
        table = []
        for R in radii:
            row = []
            for f in ratios:
                qs = [q for q, c in enumerate(cases) if c[0] == R and c[1] == round(f * R, 6)]
                row.append({"D": round(f * R, 6), "D_over_R": f,
                            "psi2_mean": float(np.nanmean(psi2[:, qs])),
                            "psi2_per_seed": [float(np.nanmean(psi2[:, q])) for q in qs],
                            "psi2_std_in_time": float(np.nanmean(np.nanstd(psi2[:, qs], axis=0))),
                            "centres_mean": float(centres[:, qs].mean())})
            means = np.array([r["psi2_mean"] for r in row])
            Ds = np.array([r["D"] for r in row])
            below = np.nonzero(means < 0.5)[0]
            Dc = None
            if len(below) and below[0] > 0:  # linear interpolation through 1/2
                i = below[0]
                Dc = float(Ds[i - 1] + (0.5 - means[i - 1]) * (Ds[i] - Ds[i - 1]) / (means[i] - means[i - 1]))
            table.append({"R": R, "D_c": Dc, "runs": row})
        return {"N": N, "L": L, "steps": steps, "transient": transient, "sample_every": every, "seeds": seeds,
                "dt": dt, "scheme": scheme,
                "coefficients": "paper preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)",
                "mask": "Algorithm 2 from the binary field outside both circles",
                "instances": n, "seconds": secs, "radii": table}
    finally:
        s.close()


def main(argv=None):
    """Dumbbell runs at the paper's coefficients; writes a JSON report."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--radii", type=float, nargs="+", default=[2.8, 3.14, 3.5])
    ap.add_argument("--ratios", type=float, nargs="+", default=[1.0, 1.2, 1.4, 1.5, 1.6, 1.7, 1.8, 1.9],
                    help="D / R values")
    ap.add_argument("--seeds", type=int, default=2)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--L", type=float, default=20.48)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--transient", type=int, default=60_000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--scheme", default="ifeuler", choices=["ifeuler", "etd1", "imex", "etdrk2", "etdrk4"])
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--report", default="dumbbell_report.json")
    a = ap.parse_args(argv)
    rep = run(a.radii, a.ratios, a.seeds, a.N, a.L, a.steps, a.transient, a.every,
              log=lambda m: print(f"[dumbbell] {m}", flush=True), scheme=a.scheme, dt=a.dt)
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f)
    print(f"[dumbbell] {rep['instances']} instances of {a.N}^2, {a.steps} steps in {rep['seconds']:.1f} s", flush=True)
    for t in rep["radii"]:
        cells = ", ".join(f"D={r['D']:.2f}: {r['psi2_mean']:.2f}" for r in t["runs"])
        dc = f"{t['D_c']:.2f}" if t["D_c"] is not None else "none"
        print(f"[dumbbell] R={t['R']:.2f}: Psi_2 {cells}; D_c {dc}", flush=True)
    return rep


if __name__ == "__main__":
    main()
