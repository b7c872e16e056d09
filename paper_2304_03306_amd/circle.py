"""Circular confinement with the paper's coefficients, several radii at once.

The circle section's set-up: the paper's preset (a, b, lambda, gamma_v,
gamma_w) = (0.5, 1.6, 9, 40, 4), the mask built by Algorithm 2 from the binary
"outside the circle" field, a box of side 40.96, random small initial fields.
Each radius is one instance of one context; after a transient the vortex
order parameter Psi, the kinetic energy and the vortex count (centres and
saddles of the velocity direction inside the circle, ttsh_vortices) are
sampled at fixed intervals, and the run reports, per radius, their mean and
spread, the most frequent vortex count and the dominant frequency of Psi(t)
(oscillating states show one), and the temporal power spectral density of
the vorticity field (eq. (PSD), accumulated on the device at every sample)
with its largest peaks.  The grid is coarser than
the paper's (its 8192^2 resolves the wall much more sharply), so the radii
at which the states change can shift.

All time stepping and measurement run in the library; the per-radius
statistics of the sampled series are host-side analysis of its output.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def _peaks(freqs, S, k=3):
    """The k largest local maxima of S(f) over f > 0, as (f, S / S_max)."""
    idx = [i for i in range(1, len(S) - 1) if S[i] >= S[i - 1] and S[i] >= S[i + 1] and freqs[i] > 0]
    idx.sort(key=lambda i: -S[i])
    top = max(S[1:]) if len(S) > 1 else 1.0
    return [(float(freqs[i]), float(S[i] / top)) for i in idx[:k]]


def run(radii, N=1024, L=40.96, steps=200_000, transient=50_000, every=200, seed=7, log=None,
        scheme: str = "ifeuler", dt: float = 0.01, psd_fmax: float = 0.1) -> dict:
    import dataclasses
    params = dataclasses.replace(W.paper_coefficients(dt=dt), scheme=scheme)
    n = len(radii)
    nsamp = (steps - transient) // every
    ts = params.dt * every  # time between samples
    freqs = np.arange(0.0, psd_fmax, 1.0 / (nsamp * ts)) if psd_fmax > 0 else np.zeros(0)
    accs = []
    if len(freqs):
        # device memory for the PSD accumulators; torch's GPU context is set up
        # before the library's, as in the other drivers that share the device
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the vorticity PSD needs a GPU visible to torch")
        accs = [torch.zeros(T.psd_buffer_len(N, len(freqs)), dtype=torch.float64, device="cuda")
                for _ in range(n)]
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
        psi = np.zeros((nsamp, n))
        energy = np.zeros((nsamp, n))
        centres = np.zeros((nsamp, n), dtype=np.int64)
        saddles = np.zeros((nsamp, n), dtype=np.int64)
        for k in range(nsamp):
            s.step(every)
            for q in range(n):
                if accs:
                    s.psd_accumulate(q, freqs, k * ts, accs[q])
                psi[k, q] = s.order(q)[0]
                sq = s.norms(q)[0]
                energy[k, q] = sq * (L / N) ** 2  # integral of |v|^2 over the box
                # nodes slower than 1e-3 of the rms speed have no defined direction
                centres[k, q], saddles[k, q] = s.vortices(q, 0.5, 1e-3 * np.sqrt(sq / (N * N)))
            if log and (k + 1) % max(1, nsamp // 10) == 0:
                log(f"sample {k + 1}/{nsamp}: Psi {np.round(psi[k], 3).tolist()}")
        s.sync()
        psd = [s.psd_finish(N, len(freqs), a) for a in accs]
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
            if psd:
                out[-1]["vorticity_psd_peaks"] = _peaks(freqs, psd[q])
                out[-1]["vorticity_psd"] = psd[q].tolist()
        return {"N": N, "L": L, "steps": steps, "transient": transient, "sample_every": every,
                "coefficients": "paper preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)",
                "mask": "Algorithm 2 from the binary outside-the-circle field",
                "seconds": secs, "radii": out, "psd_freqs": freqs.tolist(),
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
    ap.add_argument("--scheme", default="ifeuler", choices=["ifeuler", "etd1", "imex", "etdrk2", "etdrk4"])
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--psd-fmax", type=float, default=0.1,
                    help="vorticity PSD up to this frequency (cycles per unit time; 0: off)")
    ap.add_argument("--report", default="circle_report.json")
    a = ap.parse_args(argv)
    rep = run(a.radii, a.N, a.L, a.steps, a.transient, a.every, log=lambda m: print(f"[circle] {m}", flush=True),
              scheme=a.scheme, dt=a.dt, psd_fmax=a.psd_fmax)
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f)
    for r in rep["radii"]:
        print(f"[circle] R={r['R']:.2f}: Psi {r['psi_mean']:.3f} +- {r['psi_std']:.3f}, energy "
              f"{r['energy_mean']:.3g} +- {r['energy_std']:.2g}, Psi peak frequency {r['psi_peak_frequency']:.4g}, "
              f"vortex count (centres, saddles) {tuple(r['vortex_count_mode'])} in "
              f"{100 * r['vortex_count_mode_fraction']:.0f} % of samples (mean {r['centres_mean']:.2f}, "
              f"{r['saddles_mean']:.2f})", flush=True)
        if "vorticity_psd_peaks" in r:
            pk = ", ".join(f"{f:.5f} ({v:.2g})" for f, v in r["vorticity_psd_peaks"])
            print(f"[circle] R={r['R']:.2f}: vorticity PSD peaks (f, S/S_max) {pk}", flush=True)
    return rep


if __name__ == "__main__":
    main()
