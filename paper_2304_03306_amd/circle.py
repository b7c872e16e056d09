"""Circular confinement with the paper's coefficients, several radii at once.

The circle section's set-up: the paper's preset (a, b, lambda, gamma_v,
gamma_w) = (0.5, 1.6, 9, 40, 4), the mask built by Algorithm 2 from the binary
"outside the circle" field, a box of side 40.96, random small initial fields.
Each radius is one instance of one context; after a transient the vortex
order parameter Psi, the kinetic energy and the vortex count (centres and
saddles of the velocity direction inside the circle, ttsh_vortices) are
sampled at fixed intervals, and the run reports, per radius, their mean and
spread, the most frequent vortex count and the dominant frequency of Psi(t)
(oscillating states show one).  The grid is coarser than
the paper's (its 8192^2 resolves the wall much more sharply), so the radii
at which the states change can shift.

All time stepping and measurement run in the library; the per-radius
statistics of the sampled series are host-side analysis of its output.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def run(radii, N=1024, L=40.96, steps=200_000, transient=50_000, every=200, seed=7, log=None,
        scheme: str = "ifeuler", dt: float = 0.01) -> dict:
    import dataclasses
    params = dataclasses.replace(W.paper_coefficients(dt=dt), scheme=scheme)
    n = len(radii)
    s = T.Solver([N] * n, [L] * n, params, T.TTSH_FP32)
    try:
        s.option(T.TTSH_OPT_GRAPH_STEPS, every)
        for q, R in enumerate(radii):
            s.mask_from_binary(q, W.binary_outside(N, L, [(0.0, 0.0)], [R]))
            s.set_field(q, W.uniform_field(seed + q, N, 0.01, 32))
        s.tune(every)
        t0 = time.time()
        s.step(transient)
        s.sync()
        nsamp = (steps - transient) // every
        psi = np.zeros((nsamp, n))
        energy = np.zeros((nsamp, n))
        centres = np.zeros((nsamp, n), dtype=np.int64)
        saddles = np.zeros((nsamp, n), dtype=np.int64)
        for k in range(nsamp):
            s.step(every)
            for q in range(n):
                psi[k, q] = s.order(q)[0]
                sq = s.norms(q)[0]
                energy[k, q] = sq * (L / N) ** 2  # integral of |v|^2 over the box
                # nodes slower than 1e-3 of the rms speed have no defined direction
                centres[k, q], saddles[k, q] = s.vortices(q, 0.5, 1e-3 * np.sqrt(sq / (N * N)))
            if log and (k + 1) % max(1, nsamp // 10) == 0:
                log(f"sample {k + 1}/{nsamp}: Psi {np.round(psi[k], 3).tolist()}")
        s.sync()
        secs = time.time() - t0
        dt = params.dt * every
        out = []
        for q, R in enumerate(radii):
            series = psi[:, q]
            spec = np.abs(np.fft.rfft(series - series.mean())) ** 2
            freq = np.fft.rfftfreq(len(series), dt)
            f_peak = float(freq[1 + int(np.argmax(spec[1:]))]) if len(series) > 2 else 0.0
            pairs, counts = np.unique(np.stack([centres[:, q], saddles[:, q]], axis=1), axis=0, return_counts=True)
            top = pairs[int(np.argmax(counts))]
            out.append({"R": R, "psi_mean": float(series.mean()), "psi_std": float(series.std()),
                        "energy_mean": float(energy[:, q].mean()), "energy_std": float(energy[:, q].std()),
                        "psi_peak_frequency": f_peak,
                        "vortex_count_mode": [int(top[0]), int(top[1])],
                        "vortex_count_mode_fraction": float(counts.max() / nsamp),
                        "centres_mean": float(centres[:, q].mean()), "saddles_mean": float(saddles[:, q].mean())})
        return {"N": N, "L": L, "steps": steps, "transient": transient, "sample_every": every,
                "coefficients": "paper preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)",
                "mask": "Algorithm 2 from the binary outside-the-circle field",
                "seconds": secs, "radii": out,
                "psi_series": psi.tolist()}
    finally:
        s.close()


def main(argv=None):
    """Circle runs at the paper's coefficients; writes a JSON report."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--radii", type=float, nargs="+", default=[5.0, 5.2, 5.4, 5.6, 5.8, 6.0])
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--L", type=float, default=40.96)
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--transient", type=int, default=50_000)
    ap.add_argument("--every", type=int, default=200)
    ap.add_argument("--scheme", default="ifeuler", choices=["ifeuler", "etd1", "imex", "etdrk2"])
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--report", default="circle_report.json")
    a = ap.parse_args(argv)
    rep = run(a.radii, a.N, a.L, a.steps, a.transient, a.every, log=lambda m: print(f"[circle] {m}", flush=True),
              scheme=a.scheme, dt=a.dt)
    with open(a.report, "w") as f:
        json.dump(rep, f)
    for r in rep["radii"]:
        print(f"[circle] R={r['R']:.2f}: Psi {r['psi_mean']:.3f} +- {r['psi_std']:.3f}, energy "
              f"{r['energy_mean']:.3g} +- {r['energy_std']:.2g}, Psi peak frequency {r['psi_peak_frequency']:.4g}, "
              f"vortex count (centres, saddles) {tuple(r['vortex_count_mode'])} in "
              f"{100 * r['vortex_count_mode_fraction']:.0f} % of samples (mean {r['centres_mean']:.2f}, "
              f"{r['saddles_mean']:.2f})", flush=True)
    return rep


if __name__ == "__main__":
    main()
