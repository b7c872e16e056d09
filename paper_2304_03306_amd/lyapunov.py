"""Lyapunov exponents of the circular confinement at the paper's coefficients.

The circle section characterises the transition from the stationary single
vortex to the oscillating pair by the largest Lyapunov exponents, computed
with Benettin's method: independent small perturbations advanced with the
state and re-orthonormalised by a QR decomposition.  Here each radius has a
base instance and p perturbed copies, all instances of one FP64 context
advanced by the same batched step; every tau steps ttsh_lyap_qr
re-orthonormalises each radius's copies about its base on the device and
returns log R_vv.  The exponents are the averages of log R_vv / (tau dt)
over the measuring window; their spread over four consecutive sub-windows
is reported as an error estimate.  With --start-from, every radius starts from
the state settled at a larger radius (the oscillating branch), which inside
the hysteresis window follows the downward branch instead of the vortex.

The grid spacing is that of the circle runs (0.04) in a box of side 20.48, so
the radii at which the exponents cross zero can differ from the paper's.
All stepping and re-orthonormalisation run in the library; the averages are
host-side analysis of the returned logs.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import ttsh as T
from . import workloads as W


def _settled_state(R, N, L, params, steps, seed):
    """Compact FP64 state after `steps` steps from a random start at radius R
    (the starting point of the downward branch)."""
    s = T.Solver([N], [L], params, T.TTSH_FP64)
    try:
        s.mask_from_binary(0, W.binary_outside(N, L, [(0.0, 0.0)], [R]))
        s.set_field(0, W.uniform_field(seed, N, 0.01))
        s.step(steps)
        s.sync()
        return s.state(0)
    finally:
        s.close()


def run(radii, p=4, N=512, L=20.48, transient=50_000, tau=100, intervals=1000, rel_eps=1e-6, seed=3,
        log=None, dt: float = 0.01, start_from: float = 0.0) -> dict:
    params = dataclasses.replace(W.paper_coefficients(dt=dt))
    nr = len(radii)
    start = _settled_state(start_from, N, L, params, transient, seed) if start_from > 0 else None
    n = nr * (1 + p)
    s = T.Solver([N] * n, [L] * n, params, T.TTSH_FP64)
    base = [r * (1 + p) for r in range(nr)]
    pert = [[b + 1 + v for v in range(p)] for b in base]
    try:
        s.option(T.TTSH_OPT_GRAPH_STEPS, tau)
        for r, R in enumerate(radii):
            for q in [base[r]] + pert[r]:
                s.mask_from_binary(q, W.binary_outside(N, L, [(0.0, 0.0)], [R]))
            if start is None:
                s.set_field(base[r], W.uniform_field(seed + r, N, 0.01))
            else:  # every base continues the state settled at the larger radius
                s.set_state(base[r], start)
        s.tune(tau)
        t0 = time.time()
        s.step(transient)  # the copies run alongside; they are replaced below
        s.sync()
        rng = np.random.Generator(np.random.PCG64(seed + 1000))
        dst = [q for r in range(nr) for q in pert[r]]
        src = [base[r] for r in range(nr) for _ in range(p)]
        s.reseed_field(dst, src, rng.uniform(-1e-6, 1e-6, size=(len(dst), 2, N, N)))
        eps = [rel_eps * np.sqrt(s.norms(b)[0]) for b in base]
        for r in range(nr):
            s.lyap_qr(base[r], pert[r], eps[r])
        logs = np.zeros((intervals, nr, p))
        psi = np.zeros((intervals, nr))
        for j in range(intervals):
            s.step(tau)
            for r in range(nr):
                logs[j, r] = s.lyap_qr(base[r], pert[r], eps[r])
                psi[j, r] = s.order(base[r])[0]
            if log and (j + 1) % max(1, intervals // 5) == 0:
                lam = logs[: j + 1].mean(axis=0) / (tau * dt)
                log(f"interval {j + 1}/{intervals}: lambda_1 per radius {np.round(lam[:, 0], 4).tolist()}")
        s.sync()
        secs = time.time() - t0
        window = logs[intervals // 5:]  # the first fifth lets the directions converge
        lam = window.mean(axis=0) / (tau * dt)
        subs = np.array_split(window, 4)
        spread = np.std([b.mean(axis=0) / (tau * dt) for b in subs], axis=0)
        out = []
        for r, R in enumerate(radii):
            out.append({"R": R, "exponents": lam[r].tolist(), "spread": spread[r].tolist(),
                        "psi_mean": float(psi[intervals // 5:, r].mean()),
                        "psi_std": float(psi[intervals // 5:, r].std())})
        return {"N": N, "L": L, "dt": dt, "p": p, "tau": tau, "intervals": intervals, "transient": transient,
                "rel_eps": rel_eps, "precision": "FP64", "start_from": start_from or None,
                "coefficients": "paper preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)",
                "mask": "Algorithm 2 from the binary outside-the-circle field",
                "seconds": secs, "radii": out}
    finally:
        s.close()


def main(argv=None):
    """Largest Lyapunov exponents per radius (circle, paper's coefficients)."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--radii", type=float, nargs="+", default=[5.0, 5.1, 5.2, 5.3, 5.4])
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--L", type=float, default=20.48)
    ap.add_argument("--transient", type=int, default=50_000)
    ap.add_argument("--tau", type=int, default=100)
    ap.add_argument("--intervals", type=int, default=1000)
    ap.add_argument("--rel-eps", type=float, default=1e-6)
    ap.add_argument("--start-from", type=float, default=0.0,
                    help="start every radius from the state settled at this radius (0: random starts)")
    ap.add_argument("--report", default="lyapunov_report.json")
    a = ap.parse_args(argv)
    rep = run(a.radii, a.p, a.N, a.L, a.transient, a.tau, a.intervals, a.rel_eps,
              log=lambda m: print(f"[lyapunov] {m}", flush=True), start_from=a.start_from)
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f)
    print(f"[lyapunov] {len(a.radii) * (1 + a.p)} instances of {a.N}^2 (FP64), "
          f"{a.transient + a.tau * a.intervals} steps in {rep['seconds']:.1f} s", flush=True)
    for r in rep["radii"]:
        ex = ", ".join(f"{x:+.4f} +- {e:.4f}" for x, e in zip(r["exponents"], r["spread"]))
        print(f"[lyapunov] R={r['R']:.2f}: exponents {ex}; Psi {r['psi_mean']:.3f} +- {r['psi_std']:.3f}", flush=True)
    return rep


if __name__ == "__main__":
    main()
