"""Full-size workloads in the launch configuration bench.py times, against FP64
oracle states stored under tests/golden (written by make_reference_states.py,
which calls only the oracle).  The bar is the FP32 target: relative L2 error
<= 1e-5 at step 1000.  The FP64 oracle's own sensitivity at step 1000 for the
512^2 circle (a twin run started 2^-24 away) is 1.1e-7, well below it.
"""
import math
import os

import numpy as np
import pytest

from paper_2304_03306_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def ref_state(name):
    path = os.path.join(GOLDEN, f"ref_{name}_step1000.npz")
    if not os.path.exists(path):
        pytest.skip(f"reference {name} not generated")
    return np.load(path)["state"].astype(np.complex128)


def spectral_rel_l2(got, ref):
    """Relative L2 over the real field via Parseval on the compact half
    spectrum (columns m_x > 0 stand for two modes)."""
    w = np.ones(ref.shape[-1])
    w[1:] = 2.0
    return float(np.sqrt(np.sum(w * np.abs(got - ref) ** 2) / np.sum(w * np.abs(ref) ** 2)))


def build(gpu, wl, prec):
    from oracle import ttsh as O
    s = gpu.Solver([i.N for i in wl.instances], [i.L for i in wl.instances], O.workload_params(), prec)
    for q, inst in enumerate(wl.instances):
        s.mask_tanh(q, inst.centers, inst.radii, inst.xi)
        s.set_field(q, W.uniform_field(inst.seed, inst.N, 0.01, 32))
    return s


@pytest.mark.parametrize("prec", [32, 96])
def test_circle512_step1000(gpu, prec):
    print("[case] circle512 1000 steps precision", prec, flush=True)
    ref = ref_state("circle512")
    s = build(gpu, W.circle_fp32_512(), prec)
    s.step(1000)
    s.sync()
    err = spectral_rel_l2(s.state(0), ref)
    print("rel_l2", err)
    assert err <= 1e-5


def test_radius_sweep_step1000(gpu):
    print("[case] radius sweep, 64 instances, 1000 steps", flush=True)
    s = build(gpu, W.radius_sweep(), 32)
    s.step(1000)
    s.sync()
    for q, name in ((0, "sweep_R8_128"), (14, "sweep_R24_256"), (62, "sweep_R80_512")):
        err = spectral_rel_l2(s.state(q), ref_state(name))
        print(name, "rel_l2", err)
        assert err <= 1e-5, (name, err)


def test_dumbbells_step1000(gpu):
    print("[case] dumbbells, 16 x 1024^2, 1000 steps", flush=True)
    ref = ref_state("dumbbell_d40_1024")
    s = build(gpu, W.dumbbells(), 32)
    s.step(1000)
    s.sync()
    err = spectral_rel_l2(s.state(0), ref)
    print("d = 40 rel_l2", err)
    assert err <= 1e-5
    # the other end of the distance range: centre distance 80, instance 15
    err = spectral_rel_l2(s.state(15), ref_state("dumbbell_d80_1024"))
    print("d = 80 rel_l2", err)
    assert err <= 1e-5
    norms = [s.norms(q) for q in range(16)]
    # divergence of the stored FP32 spectrum: rounding of a projected FP64 update
    assert all(np.isfinite(n[0]) and n[3] < 1e-6 * np.sqrt(n[0]) for n in norms)


def test_hysteresis_scan_runs_all_stages(gpu):
    """Two short stages of the batched sweep with continuation: every
    instance's order parameter is recorded after each stage, finite and in
    the parameter's range; the smallest radius (one vortex) orders more than
    the largest (many)."""
    from paper_2304_03306_amd import sweep
    print("[case] sweep 2 stages x 400 steps", flush=True)
    rep = sweep.run(2, 400, tune=False)
    up, down = np.array(rep["psi_up"]), np.array(rep["psi_down"])
    assert up.shape == (2, 32) and down.shape == (2, 32)
    assert np.isfinite(up).all() and np.isfinite(down).all()
    assert (np.abs(up) <= 1.0 + 1e-12).all() and (np.abs(down) <= 1.0 + 1e-12).all()
    assert rep["radii"][0] == 8.0 and abs(rep["radii"][-1] - 80.0) < 1e-12


def test_circle_driver_short_run(gpu):
    """The paper-preset circle driver on two small radii for a few thousand
    steps: finite order parameters and energies, one record per radius."""
    from paper_2304_03306_amd import circle
    print("[case] circle driver 256^2 x 2 radii", flush=True)
    rep = circle.run([5.2, 5.6], N=256, L=40.96, steps=3000, transient=1000, every=200)
    assert [r["R"] for r in rep["radii"]] == [5.2, 5.6]
    for r in rep["radii"]:
        assert np.isfinite(r["psi_mean"]) and np.isfinite(r["energy_mean"]) and r["energy_mean"] >= 0
    assert np.array(rep["psi_series"]).shape == (10, 2)
    # the vorticity PSD on the record's frequency grid, non-negative
    assert len(rep["psd_freqs"]) >= 1
    for r in rep["radii"]:
        assert len(r["vorticity_psd"]) == len(rep["psd_freqs"]) and min(r["vorticity_psd"]) >= 0


def test_dumbbell_driver_short_run(gpu):
    """The dumbbell driver on one radius and two distances: Psi_2 in [0, 1]
    for every cell, one row per distance."""
    from paper_2304_03306_amd import dumbbell
    print("[case] dumbbell driver 256^2 x 2 distances", flush=True)
    rep = dumbbell.run([3.14], [1.2, 1.8], seeds=1, N=256, L=20.48, steps=3000, transient=1000, every=500)
    rows = rep["radii"][0]["runs"]
    assert [r["D_over_R"] for r in rows] == [1.2, 1.8]
    for r in rows:
        assert 0.0 <= r["psi2_mean"] <= 1.0


def test_hysteresis_driver_short_run(gpu):
    """The ramp driver on three radii for three short stages: both ramps
    recorded at every stage, Psi finite."""
    from paper_2304_03306_amd import hysteresis
    print("[case] hysteresis driver 256^2 x 3 radii", flush=True)
    rep = hysteresis.run([5.2, 5.3, 5.4], steps=1000, every=100, N=256, L=20.48, noise=1e-3)
    assert len(rep["record"]) == 3 and len(rep["radii"]) == 3
    for r in rep["radii"]:
        assert np.isfinite(r["up_psi"]) and np.isfinite(r["down_psi"])


def test_lyapunov_driver_short_run(gpu):
    """The Lyapunov driver on one radius, two copies, a few intervals: two
    finite exponents."""
    from paper_2304_03306_amd import lyapunov
    print("[case] lyapunov driver 256^2 x 1 radius", flush=True)
    rep = lyapunov.run([5.2], p=2, N=256, L=20.48, transient=500, tau=50, intervals=10)
    ex = rep["radii"][0]["exponents"]
    assert len(ex) == 2 and all(np.isfinite(ex))


@pytest.mark.parametrize("prec", [32])
def test_diagnostics_match_oracle_1024(gpu, prec):
    """At the circle driver's size (1024^2, the reductions at their full
    spread of 256 workgroups): Psi, Psi_2 (half-planes and two-chamber disks)
    and the vortex count of a paper-preset state in a circle of radius 5.6
    (Algorithm 2 mask, 3000 steps from a seeded start) equal the oracle's on
    the same real-space fields."""
    from oracle import ttsh as O
    print("[case] diagnostics 1024^2 vs oracle", flush=True)
    N, L = 1024, 40.96
    s = gpu.Solver([N], [L], W.paper_coefficients(), prec)
    try:
        s.mask_from_binary(0, W.binary_outside(N, L, [(0.0, 0.0)], [5.6]))
        s.set_field(0, W.uniform_field(12, N, 0.01, prec))
        s.step(3000)
        s.sync()
        vh = O.from_compact(s.state(0), N)
        kx, ky, _, _ = O.grid(N, L)
        v = O.field(vh)
        w = O.field(O.vorticity_hat(vh, kx, ky)[None])[0]
        for cen in ((0.0, 0.0), (0.3, -0.2)):
            psi, psi2 = s.order(0, cen)
            assert abs(psi - O.vortex_order(v, L, cen)) < 1e-12
            assert abs(psi2 - O.vortex_order2(w, L, cen[0])) < 1e-12
            for D in (3.0, 5.0):
                assert abs(s.order_dumbbell(0, D, cen) - O.vortex_order2(w, L, cen[0], D=D, center_y=cen[1])) < 1e-12
        vmin = 1e-3 * math.sqrt(s.norms(0)[0] / (N * N))
        K = s.mask(0)
        # on the real-space field the library computes (its own FP64 transform)
        assert s.vortices(0, 0.5, vmin) == O.vortex_count(s.field(0), K, 0.5, vmin)
    finally:
        s.close()
