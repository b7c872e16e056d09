"""Pins of the FP64 oracle against what the paper and the mathematics fix
(closed forms, invariants, brute force on tiny grids, symmetries).  CPU only.

Each pin names the passage it follows.  Numbers written into the tests are
derived by hand from the model, not by calling the oracle's own formulas:
for the workload coefficients (alpha, beta, Gamma0, Gamma2) = (-1, 1, -1, 1)
the linear symbol is L(k) = 1 + k^2 - k^4, so L(0) = 1, L = 5/4 at k^2 = 1/2
(its maximum) and L = 0 at k^2 = (1 + sqrt 5)/2; for the paper's a = 0.5,
L = a - (1 - k^2)^2 gives L = 0.5 at k = 1 and -0.5 at k = 0.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import ttsh as O
from paper_2304_03306_amd import workloads as W

PHI = (1.0 + math.sqrt(5.0)) / 2.0


def zero_nl(p):
    return dataclasses.replace(p, beta=0.0, lambda0=0.0, lambda1=0.0, gamma_v=0.0, gamma_w=0.0)


def mode_field(N, L, mx, my, amp=1.0, phase=0.3):
    """Divergence-free single-mode velocity from psi = amp cos(k.x + phase)."""
    x, y = O.node_coords(N, L)
    kx, ky = 2 * math.pi * mx / L, 2 * math.pi * my / L
    s = -amp * np.sin(kx * x + ky * y + phase)
    return np.stack([ky * s, -kx * s])  # (d_y psi, -d_x psi)


def both_forms(v0, K, p, L, n):
    """Run Algorithm 1 and the velocity form n steps; return both spectra."""
    N = v0.shape[-1]
    kx, ky, k2, _ = O.grid(N, L)
    v, w = O.alg1_init(v0, L)
    vh = O.project_field(v0, L)
    for _ in range(n):
        v, w = O.alg1_step(v, w, K, p, L)
        vh = O.velocity_step(vh, K, p, L)
    return O.dft2(v), vh


# ---- P1/P2: the DFT of Appendix C ------------------------------------------------
@pytest.mark.parametrize("N", [4, 8, 16])
def test_dft_matches_bruteforce(N):
    rng = np.random.default_rng(N)
    f = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    assert np.abs(O.dft2(f) - O.dft2_bruteforce(f, -1)).max() < 1e-13
    assert np.abs(O.idft2(f) - O.dft2_bruteforce(f, +1)).max() < 1e-13


def test_parseval_and_roundtrip():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((64, 64))
    F = O.dft2(f)
    assert abs(np.sum(np.abs(F) ** 2) - np.sum(f * f)) < 1e-12 * np.sum(f * f)
    assert np.abs(O.idft2(F) - f).max() < 1e-14


def test_dft_sign_convention():
    # f = cos(2 pi x / N) on index grid: forward transform puts N/2 at m = +1 and -1
    N = 8
    j = np.arange(N)
    f = np.exp(2j * math.pi * 1 * j / N)[None, :] * np.ones((N, 1))
    F = O.dft2(f)
    assert abs(F[0, 1] - N) < 1e-12 and np.abs(F).sum() - N < 1e-12


# ---- P3/P4: linear growth and decay of a single Fourier mode --------------------------
@pytest.mark.parametrize("scheme", ["ifeuler", "etd1", "imex"])
@pytest.mark.parametrize("k2,rate", [(0.5, 1.25), (PHI, 0.0), (2.0, 1.0 + 2.0 - 4.0)])
def test_single_mode_growth_rate(scheme, k2, rate):
    N, n = 16, 200
    p = dataclasses.replace(zero_nl(O.workload_params()), scheme=scheme)
    # mode m = (1, 1) has k^2 = 2 (2 pi / L)^2; choose L to hit k2
    L = 2 * math.pi * math.sqrt(2.0 / k2)
    v0 = mode_field(N, L, 1, 1)
    a, b = both_forms(v0, np.zeros((N, N)), p, L, n)
    for vh in (a, b):
        ratio = abs(vh[1, 1, 1]) / abs(O.project_field(v0, L)[1, 1, 1])
        got = math.log(ratio) / (n * p.dt)
        want = rate if scheme != "imex" else -math.log(1.0 - p.dt * rate) / p.dt
        assert abs(got - want) < 1e-11, (got, want)


def test_paper_symbol_values():
    p = zero_nl(O.paper_params())
    N, n = 16, 100
    for k2, rate in ((1.0, 0.5), (0.0, -0.5)):
        if k2 == 0.0:
            v0 = np.ones((2, N, N)) * np.array([0.3, -0.2])[:, None, None]
            L = 10.0
            vh = O.run_velocity(O.project_field(v0, L), np.zeros((N, N)), p, L, n)
            got = math.log(abs(vh[0, 0, 0].real) / (0.3 * N)) / (n * p.dt)
        else:
            L = 2 * math.pi * math.sqrt(2.0)
            v0 = mode_field(N, L, 1, 1)
            vh = O.run_velocity(O.project_field(v0, L), np.zeros((N, N)), p, L, n)
            got = math.log(abs(vh[1, 1, 1]) / abs(O.project_field(v0, L)[1, 1, 1])) / (n * p.dt)
        assert abs(got - rate) < 1e-11


# ---- P5: single-shell cellular flow: advection vanishes exactly ------------------------
def test_cellular_flow_advection_free():
    N, L, n = 32, 40.0, 60
    p = dataclasses.replace(zero_nl(O.workload_params()), lambda0=3.0)
    v0 = mode_field(N, L, 3, 0, 0.7, 0.1) + mode_field(N, L, 0, 3, 0.7, -0.4)
    k2 = (2 * math.pi * 3 / L) ** 2
    growth = math.exp((1.0 + k2 - k2 * k2) * p.dt * n)
    a, b = both_forms(v0, np.zeros((N, N)), p, L, n)
    ref = O.project_field(v0, L) * growth
    for vh in (a, b):
        assert np.abs(vh - ref).max() < 1e-12 * np.abs(ref).max()


# ---- P6: shear mode, cubic term and vanishing advection ------------------------------------
def test_shear_mode_cubic_term():
    N, L, m, A = 32, 32.0, 2, 0.8
    p = dataclasses.replace(O.workload_params(), gamma_v=0.0)  # beta = 1, lambda0 = 3
    x, y = O.node_coords(N, L)
    th = 2 * math.pi * m * (y + L / 2) / L
    v0 = np.stack([A * np.cos(th), np.zeros((N, N))])
    a, b = both_forms(v0, np.zeros((N, N)), p, L, 1)
    k1 = (2 * math.pi * m / L) ** 2
    k3 = (2 * math.pi * 3 * m / L) ** 2
    E1 = math.exp((1 + k1 - k1 * k1) * p.dt)
    E3 = math.exp((1 + k3 - k3 * k3) * p.dt)
    # cos^3 = (3 cos th + cos 3 th)/4; unitary DFT of c cos(q y) has N c / 2 at m_y = +-q
    want1 = E1 * (A - p.dt * p.beta * 0.75 * A ** 3) * N / 2
    want3 = E3 * (-p.dt * p.beta * 0.25 * A ** 3) * N / 2
    for vh in (a, b):
        assert abs(abs(vh[0, m, 0]) - abs(want1)) < 1e-12
        assert abs(abs(vh[0, 3 * m, 0]) - abs(want3)) < 1e-12
        assert np.abs(vh[1]).max() < 1e-12  # no y velocity is created


# ---- Galilean shift: advection sign and strength ---------------------------------------
@pytest.mark.parametrize("lam", [3.0, -2.0])
def test_advection_by_uniform_flow(lam):
    """alpha = beta = 0, K = 0: v = (U, 0) + (0, a cos(k x)).  The forcing is
    exactly -lambda0 U d_x u, so the discrete scheme maps the mode by
    E(k) (1 - i lambda0 U k dt) per step (u_hat(k) multiplies by -i k U)."""
    N, L, m, U, n = 32, 32.0, 3, 0.7, 40
    p = dataclasses.replace(O.workload_params(), alpha=0.0, beta=0.0, gamma_v=0.0, lambda0=lam)
    x, y = O.node_coords(N, L)
    k = 2 * math.pi * m / L
    v0 = np.stack([np.full((N, N), U), 0.4 * np.cos(k * (x + L / 2))])
    a, b = both_forms(v0, np.zeros((N, N)), p, L, n)
    E = math.exp((k * k - k ** 4) * p.dt)  # L = k^2 - k^4 once alpha = 0
    mult = E * complex(1.0, -lam * U * k * p.dt)
    v0h = O.project_field(v0, L)
    for vh in (a, b):
        assert abs(vh[1, 0, m] - v0h[1, 0, m] * mult ** n) < 1e-12 * abs(v0h[1, 0, m])
        assert abs(vh[0, 0, 0] - v0h[0, 0, 0]) < 1e-12 * abs(v0h[0, 0, 0])


# ---- P7: uniform state, fixed point of the discrete map (eq. (7)) ------------------------
def test_uniform_state_fixed_point():
    p = O.workload_params()
    N, L = 8, 8.0
    c = 0.3
    vh = O.project_field(np.stack([np.full((N, N), c), np.zeros((N, N))]), L)
    e = 1.010050167084168  # exp(0.01) = exp(-alpha dt)
    for _ in range(3000):
        vh = O.velocity_step(vh, np.zeros((N, N)), p, L)
        c = e * (c - 0.01 * c ** 3)
    assert abs(vh[0, 0, 0].real / N - c) < 1e-14
    # |v|^2 -> (1 - exp(alpha dt)) / (beta dt) = 0.995016625083195...
    assert abs(c * c - 0.995016625083195) < 1e-12
    v, w = O.alg1_init(np.stack([np.full((N, N), 0.3), np.zeros((N, N))]), L)
    for _ in range(3000):
        v, w = O.alg1_step(v, w, np.zeros((N, N)), p, L)
    assert abs(v[0, 0, 0] ** 2 - 0.995016625083195) < 1e-12


# ---- P8: constant mask ------------------------------------------------------------------------
def test_constant_mask_damping():
    N, L, cst = 16, 20.0, 0.37
    p = dataclasses.replace(zero_nl(O.workload_params()), gamma_v=100.0)
    v0 = W.uniform_field(3, N, 0.5)
    vh0 = O.project_field(v0, L)
    _, _, k2, _ = O.grid(N, L)
    E = np.exp((1 + k2 - k2 * k2) * p.dt)
    a, b = both_forms(v0, np.full((N, N), cst), p, L, 1)
    for vh in (a, b):
        assert np.abs(vh - E * (1 - 100.0 * cst * p.dt) * vh0).max() < 1e-13


def test_constant_mask_vorticity_damping():
    """-gamma_w K omega acts on k != 0 only (omega has no k = 0 part)."""
    N, L, cst = 16, 20.0, 0.5
    p = dataclasses.replace(zero_nl(O.workload_params()), gamma_w=4.0)
    v0 = W.uniform_field(4, N, 0.5)
    vh0 = O.project_field(v0, L)
    _, _, k2, _ = O.grid(N, L)
    E = np.exp((1 + k2 - k2 * k2) * p.dt)
    want = E * (1 - 4.0 * cst * p.dt) * vh0
    want[:, 0, 0] = E[0, 0] * vh0[:, 0, 0]
    a, b = both_forms(v0, np.full((N, N), cst), p, L, 1)
    for vh in (a, b):
        assert np.abs(vh - want).max() < 1e-13


# ---- P9-P11: invariants -------------------------------------------------------------------------
def test_divergence_free_real_and_mean_vorticity():
    N, L = 32, 16.0
    p = O.paper_params()
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v, w = O.alg1_init(W.uniform_field(5, N, 0.5), L)
    for _ in range(20):
        v, w = O.alg1_step(v, w, K, p, L)
    kx, ky, _, _ = O.grid(N, L)
    vh = O.dft2(v)
    assert np.abs(kx * vh[0] + ky * vh[1]).max() < 1e-12 * np.abs(vh).max()
    assert w[0, 0] == 0
    assert np.abs(O.idft2(w).imag).max() < 1e-15 * np.abs(w).max() * N


def test_velocity_form_stays_divergence_free():
    """Algorithm 1 derives v from the stream function every step, so the
    velocity must stay divergence-free over long runs even where L(k) > 0
    would amplify any divergent rounding error by e^{L t} (here e^{1.25 * 30})."""
    N, L = 32, 32.0
    K = O.mask_tanh(N, L, [(0, 0)], [10.0], 0.5)
    p = O.workload_params()
    vh = O.project_field(W.uniform_field(13, N, 0.01), L)
    kx, ky, _, _ = O.grid(N, L)
    for _ in range(3000):
        vh = O.velocity_step(vh, K, p, L)
    assert np.abs(kx * vh[0] + ky * vh[1]).max() < 1e-13 * np.abs(vh).max()


def test_projection_idempotent_and_gradient_free():
    N, L = 32, 16.0
    kx, ky, k2, _ = O.grid(N, L)
    vh = O.project_field(W.uniform_field(6, N, 1.0), L)
    assert np.abs(O.leray(vh, kx, ky, k2) - vh).max() < 1e-13
    g = O.dft2(np.random.default_rng(2).standard_normal((N, N)))
    grad = np.stack([1j * kx * g, 1j * ky * g])
    pg = O.leray(grad, kx, ky, k2)
    pg[:, 0, 0] = 0
    assert np.abs(pg).max() < 1e-12 * np.abs(grad).max()


def test_lambda1_is_a_no_op():
    N, L = 32, 16.0
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    vh = O.project_field(W.uniform_field(7, N, 0.5), L)
    p0 = O.workload_params()
    p1 = dataclasses.replace(p0, lambda1=2.5)
    a = O.run_velocity(vh, K, p0, L, 10)
    b = O.run_velocity(vh, K, p1, L, 10)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_dealias_cutoff_is_strict():
    """1/2 rule: m^2 > (N/4)^2 removed, m^2 = (N/4)^2 kept (Algorithm 1)."""
    N = 16
    keep = O.dealias_keep(N)
    M = N // 4
    assert keep[0, M] and keep[M, 0] and keep[-M, 0] and keep[0, -M]
    assert not keep[1, M] and not keep[M, 1]
    assert keep.sum() == sum(1 for a in range(-8, 8) for b in range(-8, 8) if a * a + b * b <= 16)


# ---- P12: Algorithm 1 (vorticity, convective) equals the velocity form -------------------------
@pytest.mark.parametrize("params", ["paper", "workload"])
def test_alg1_equals_velocity_form(params):
    N, L = 32, 24.0
    p = O.paper_params() if params == "paper" else O.workload_params()
    K = O.mask_tanh(N, L, [(0, 0)], [7.0], 0.5)
    a, b = both_forms(W.uniform_field(8, N, 0.6), K, p, L, 10)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


# ---- P13/P14: symmetry ------------------------------------------------------------------------------
@pytest.mark.parametrize("g", ["rot", "refl", "transpose"])
def test_d4_equivariance(g):
    N, L = 32, 32.0
    p = O.paper_params()
    K = O.mask_tanh(N, L, [(0, 0)], [9.0], 0.5)
    act = {"rot": O.rotate90, "refl": O.reflect_x, "transpose": O.transpose_xy}[g]
    # the mask is symmetric under the group (as a scalar field)
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    Kg = {"rot": K[(N - J) % N, I], "refl": K[:, (N - np.arange(N)) % N], "transpose": K.T}[g]
    assert np.array_equal(Kg, K)
    v0 = O.field(O.project_field(W.uniform_field(9, N, 0.5), L))
    a = O.field(O.run_velocity(O.project_field(v0, L), K, p, L, 10))
    b = O.field(O.run_velocity(O.project_field(act(v0), L), K, p, L, 10))
    assert np.abs(act(a) - b).max() < 1e-12 * np.abs(a).max()


def test_translation_equivariance():
    N, L, sh = 32, 32.0, (3, -5)
    p = O.paper_params()
    K = O.mask_tanh(N, L, [(0, 0)], [9.0], 0.5)
    v0 = W.uniform_field(10, N, 0.5)
    a = O.field(O.run_velocity(O.project_field(v0, L), K, p, L, 5))
    b = O.field(O.run_velocity(O.project_field(np.roll(v0, sh, (1, 2)), L), np.roll(K, sh, (0, 1)), p, L, 5))
    assert np.abs(np.roll(a, sh, (1, 2)) - b).max() < 1e-12 * np.abs(a).max()


# ---- P15: first order in time ---------------------------------------------------------------------
def test_first_order_convergence():
    N, L, T_end = 16, 16.0, 0.4
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v0 = O.project_field(W.uniform_field(11, N, 0.8), L)
    out = {}
    for dt in (0.02, 0.01, 0.005, 0.0025):
        p = dataclasses.replace(O.workload_params(), dt=dt, gamma_v=10.0)
        out[dt] = O.run_velocity(v0, K, p, L, int(round(T_end / dt)))
    e1 = np.abs(out[0.02] - out[0.0025]).max()
    e2 = np.abs(out[0.01] - out[0.0025]).max()
    e3 = np.abs(out[0.005] - out[0.0025]).max()
    # errors against the finest run of a first-order method: (7, 3, 1) x c
    assert abs(e1 / e3 - 7.0) < 0.4 and abs(e2 / e3 - 3.0) < 0.2


# ---- P16/P17: masks ----------------------------------------------------------------------------------
def test_alg2_mask_properties():
    N, L = 64, 64.0
    Kn = W.binary_outside(N, L, [(0, 0)], [12.0])
    K = O.mask_alg2(Kn)
    assert (K >= 0).all()
    _, _, _, m2 = O.grid(N, L)
    Kh = O.dft2(K)
    assert np.abs(Kh[m2 > (N // 4) ** 2]).max() < 1e-12 * np.abs(Kh).max()
    # mirror symmetry of the disk about the centre node
    assert np.abs(K - K[:, (N - np.arange(N)) % N]).max() < 1e-13
    assert K[N // 2, N // 2] < 0.05 and K[0, 0] > 0.9


def test_alg2_on_band_limited_input_is_square():
    """If the input has no modes above (N/8)^2, the cutoff does nothing and
    Algorithm 2 returns the square of the input."""
    N, L = 32, 32.0
    x, y = O.node_coords(N, L)
    f = 0.5 + 0.3 * np.cos(2 * math.pi * 2 * x / L) * np.sin(2 * math.pi * 3 * y / L)
    assert np.abs(O.mask_alg2(f) - f * f).max() < 1e-14


def test_tanh_mask_values():
    N, L = 64, 64.0
    K = O.mask_tanh(N, L, [(0, 0)], [8.0], 0.5)
    # node at (x, y) = (8, 0) lies on the circle: K = 1/2 exactly
    assert K[N // 2, N // 2 + 8] == 0.5
    # centre: (1 + tanh(-16))/2
    assert abs(K[N // 2, N // 2] - 0.5 * (1 + math.tanh(-16.0))) < 1e-22
    assert abs(K[0, 0] - 1.0) < 1e-15
    D = O.mask_tanh(N, L, [(-4, 0), (4, 0)], [8.0, 8.0], 0.5)
    A = O.mask_tanh(N, L, [(-4, 0)], [8.0], 0.5)
    B = O.mask_tanh(N, L, [(4, 0)], [8.0], 0.5)
    assert np.array_equal(D, A * B)


# ---- compact layout and diagnostics ----------------------------------------------------------------
def test_compact_roundtrip():
    N, L = 32, 16.0
    vh = O.project_field(W.uniform_field(12, N, 1.0), L)
    assert np.abs(O.from_compact(O.to_compact(vh), N) - vh).max() < 1e-15


def test_vortex_order_parameter_limits():
    N, L = 64, 64.0
    x, y = O.node_coords(N, L)
    r = np.sqrt(x * x + y * y) + 1e-300
    az = np.stack([-y / r, x / r])
    az[:, N // 2, N // 2] = 0
    assert abs(O.vortex_order(az, L) - 1.0) < 1e-12
    # a uniform flow inside a disk has mean |e_theta . v| / |v| = 2/pi: Psi = 0
    disk = (r < L / 4).astype(float)
    uni = np.stack([disk, np.zeros((N, N))])
    assert abs(O.vortex_order(uni, L)) < 0.01


# ---- continuation between grids -----------------------------------------------------
def test_resample_preserves_band_limited_field():
    """A field inside the smaller grid's 1/2-rule disk is reproduced exactly
    (as a physical field sampled on the other grid) in both directions."""
    Ns, Nd, L = 32, 64, 20.0
    vh = O.project_field(W.uniform_field(21, Ns, 1.0), L)
    up = O.resample(vh, Nd)
    xs = np.arange(Ns) * L / Ns
    xd = np.arange(Nd) * L / Nd
    # evaluate both spectra as trigonometric sums at the coarse nodes
    f_s = O.field(vh)
    f_d = O.field(up)
    assert np.abs(f_d[:, ::2, ::2] - f_s).max() < 1e-12
    back = O.resample(up, Ns)
    assert np.abs(back - vh).max() < 1e-12
    # truncation drops exactly the modes outside the coarse disk
    vh64 = O.project_field(W.uniform_field(22, Nd, 1.0), L)
    down = O.resample(vh64, Ns)
    keep = O.dealias_keep(Ns)
    assert np.abs(down[:, ~keep]).max() == 0


def test_vortex_order2_limits():
    """Psi_2 (two-chamber section): two co-rotating Gaussian vortices give 1,
    counter-rotating ones 0, whatever their (unequal) strengths and the
    background noise below their peaks."""
    N, L = 64, 64.0
    x, y = O.node_coords(N, L)
    bump = lambda cx, a: a * np.exp(-((x - cx) ** 2 + y ** 2) / 20.0)
    rng = np.random.default_rng(0)
    noise = 1e-3 * rng.standard_normal((N, N))
    w_same = bump(-16.0, 1.0) + bump(16.0, 0.7) + noise
    w_opp = bump(-16.0, 1.0) + bump(16.0, -0.7) + noise
    assert abs(O.vortex_order2(w_same, L) - 1.0) < 1e-12
    assert O.vortex_order2(w_opp, L) < 0.2 and abs(O.vortex_order2(w_opp, L) - 0.3 / 1.7) < 5e-3
    # the split decides which peaks compete: past the right vortex the right
    # side holds only noise, so Psi_2 is ~1 whatever the vortices' signs
    assert O.vortex_order2(w_opp, L, split_x=30.0) > 0.99
    # the paper's regions (the disks of radius D/2 about the cavity centres
    # -+D/2): a stronger spike outside both disks (near the far wall) does not
    # compete there, while the half-planes pick it up
    spike = np.zeros((N, N))
    spike[N // 2 + 20, 16] = -5.0  # (x, y) = (-16, 20): in the left half, outside the left disk
    assert (x[N // 2 + 20, 16], y[N // 2 + 20, 16]) == (-16.0, 20.0)
    assert abs(O.vortex_order2(w_same + spike, L, D=32.0) - 1.0) < 1e-12
    assert O.vortex_order2(w_same + spike, L) < 0.9
    assert abs(O.vortex_order2(w_opp + spike, L, D=32.0) - 0.3 / 1.7) < 5e-3


# ---- second-order exponential Runge-Kutta (ETD2RK, Cox and Matthews 2002) -----------------
def test_phi_functions_match_high_precision():
    """phi_1(z) = (e^z - 1)/z and phi_2(z) = (e^z - 1 - z)/z^2 against 40-digit
    evaluations, across the series / closed-form switch and the stiff range."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    z = np.array([0.0, 1e-12, -3e-6, 4e-3, -9.9e-3, 1.0e-2, -1.5e-2, 0.3, -2.0, 1.25, -80.0, -5e3])
    p1, p2 = O.phi_functions(z)
    for zi, a, b in zip(z, p1, p2):
        if zi == 0.0:
            w1, w2 = 1.0, 0.5
        else:
            q = mpmath.mpf(float(zi))
            w1, w2 = float(mpmath.expm1(q) / q), float((mpmath.expm1(q) - q) / q ** 2)
        assert abs(a - w1) <= 1e-15 * abs(w1) and abs(b - w2) <= 1e-13 * abs(w2), (zi, a, w1, b, w2)


@pytest.mark.parametrize("k2,rate", [(0.5, 1.25), (PHI, 0.0), (2.0, 1.0 + 2.0 - 4.0)])
def test_etdrk2_linear_modes_are_exact(k2, rate):
    """With the forcing switched off both stages reduce to e^{L dt}: the
    measured rate of a single mode is L(k) to round-off (P3/P4)."""
    N, n = 16, 200
    p = dataclasses.replace(zero_nl(O.workload_params()), scheme="etdrk2")
    L = 2 * math.pi * math.sqrt(2.0 / k2)
    v0 = O.project_field(mode_field(N, L, 1, 1), L)
    vh = O.run_velocity(v0, np.zeros((N, N)), p, L, n)
    got = math.log(abs(vh[1, 1, 1]) / abs(v0[1, 1, 1])) / (n * p.dt)
    assert abs(got - rate) < 1e-11, (got, rate)


@pytest.mark.parametrize("preset", ["workload", "paper"])
def test_etdrk2_second_order_convergence(preset):
    """Errors against the finest run scale as dt^2: for dt = 8h, 4h, 2h against
    h the differences are c (64 - 1, 16 - 1, 4 - 1) h^2, ratios 21 and 5 (a
    dropped or mis-weighted second stage falls back to first order: 7 and 3).
    The paper preset exercises the gamma_w (vorticity) source as well."""
    N, L = 16, 16.0
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v0 = O.project_field(W.uniform_field(11, N, 0.8), L)
    if preset == "workload":
        base, T_end, dts = dataclasses.replace(O.workload_params(), gamma_v=10.0), 0.4, (0.01, 0.005, 0.0025, 0.00125)
    else:
        base, T_end, dts = dataclasses.replace(O.paper_params(), gamma_v=10.0, gamma_w=2.0), 0.2, (0.004, 0.002, 0.001, 0.0005)
    out = {dt: O.run_velocity(v0, K, dataclasses.replace(base, dt=dt, scheme="etdrk2"), L, int(round(T_end / dt)))
           for dt in dts}
    e = [np.abs(out[dt] - out[dts[-1]]).max() for dt in dts[:3]]
    assert abs(e[0] / e[2] - 21.0) < 1.5 and abs(e[1] / e[2] - 5.0) < 0.2, e


def test_etdrk2_solves_the_same_equation_as_algorithm_1():
    """ETD2RK and the paper's first-order scheme converge to the same
    solution: ETD2RK at dt agrees with the Richardson extrapolation
    2 u_ifeuler(dt/2) - u_ifeuler(dt) (second-order accurate) to within 2 % of
    the difference between the two schemes at dt."""
    N, L, T_end, dt = 16, 16.0, 0.4, 0.0025
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v0 = O.project_field(W.uniform_field(11, N, 0.8), L)
    base = dataclasses.replace(O.workload_params(), gamma_v=10.0)
    etd = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt, scheme="etdrk2"), L, int(round(T_end / dt)))
    if1 = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt), L, int(round(T_end / dt)))
    if2 = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt / 2), L, int(round(2 * T_end / dt)))
    assert np.abs(etd - (2 * if2 - if1)).max() < 0.02 * np.abs(etd - if1).max()


def test_etdrk2_stays_divergence_free_and_hermitian():
    N, L = 32, 32.0
    K = O.mask_tanh(N, L, [(0, 0)], [10.0], 0.5)
    p = dataclasses.replace(O.workload_params(), scheme="etdrk2")
    vh = O.project_field(W.uniform_field(13, N, 0.01), L)
    kx, ky, _, _ = O.grid(N, L)
    for _ in range(1500):
        vh = O.run_velocity(vh, K, p, L, 1)
    assert np.abs(kx * vh[0] + ky * vh[1]).max() < 1e-13 * np.abs(vh).max()
    assert np.array_equal(vh, np.conj(O.reflect(vh)))


# ---- vortex counting (topological charge of the velocity direction field) --------------------
def test_vortex_count_closed_forms():
    """Index of the direction field of v: +1 at vortex centres of either sense,
    -1 at saddles.  psi = sin x sin y on the periodic box has four centres and
    four saddles (Poincare-Hopf: the indices sum to zero on the torus); a
    localised vortex and a saddle inside a disk count (1, 0) and (0, 1);
    a uniform flow has none; reversing v changes nothing."""
    N, L = 64, 2 * math.pi
    x, y = O.node_coords(N, L)
    x, y = x + 0.013, y + 0.021  # critical points off the nodes
    cell = np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
    zero = np.zeros((N, N))
    assert O.vortex_count(cell, zero, 0.5, 0.0) == (4, 4)
    assert O.vortex_count(-cell, zero, 0.5, 0.0) == (4, 4)
    r2 = (x - 0.3) ** 2 + (y + 0.2) ** 2
    disk = (r2 > 2.0).astype(float)
    g = np.exp(-r2 / 0.5)
    vort = np.stack([-(y + 0.2) * g, (x - 0.3) * g])
    assert O.vortex_count(vort, disk, 0.5, 1e-12) == (1, 0)
    assert O.vortex_count(-vort, disk, 0.5, 1e-12) == (1, 0)
    assert O.vortex_count(np.stack([x - 0.3, -(y + 0.2)]), disk, 0.5, 1e-12) == (0, 1)
    assert O.vortex_count(np.stack([np.ones((N, N)), 0.3 * np.ones((N, N))]), zero, 0.5, 0.0) == (0, 0)
    # cells touching the excluded region (mask or slow nodes) do not count
    assert O.vortex_count(vort, np.ones((N, N)), 0.5, 1e-12) == (0, 0)
    assert O.vortex_count(vort, disk, 0.5, 10.0) == (0, 0)


def test_vortex_count_defect_on_a_node():
    """A vortex centred exactly on a node (v = 0 there, as for a symmetric
    vortex in a circle centred on a node) is counted once, from the ring of
    the node's eight neighbours; so is a saddle on a node."""
    N, L = 64, 32.0
    x, y = O.node_coords(N, L)
    r2 = x * x + y * y
    disk = (r2 > 100.0).astype(float)
    g = np.exp(-r2 / 20.0)
    vort = np.stack([-y * g, x * g])
    assert vort[:, N // 2, N // 2].tolist() == [0.0, 0.0]
    assert O.vortex_count(vort, disk, 0.5, 1e-12) == (1, 0)
    assert O.vortex_count(np.stack([x, -y]), disk, 0.5, 1e-12) == (0, 1)


# ---- Lyapunov exponents (Benettin's method with QR re-orthonormalisation) --------------------
def test_lyap_inner_is_the_real_space_inner_product():
    """The weighted compact inner product equals sum_x v_a . v_b over the grid
    nodes of the two real fields (Parseval with the unitary DFT): a dropped
    weight on the m_x > 0 columns or a conjugation slip fails it."""
    N, L = 32, 20.0
    a = O.project_field(W.uniform_field(1, N, 1.0), L)
    b = O.project_field(W.uniform_field(2, N, 1.0), L)
    va, vb = O.field(a), O.field(b)
    ca, cb = O.to_compact(a), O.to_compact(b)
    assert abs(O.lyap_inner(ca, cb, N) - float(np.sum(va * vb))) < 1e-12 * float(np.sum(va * va))
    assert abs(O.lyap_inner(ca, ca, N) - float(np.sum(va * va))) < 1e-12 * float(np.sum(va * va))


def test_lyapunov_qr_orthonormal_and_triangular():
    """After lyapunov_qr the deviations (X_i - X_0)/eps are orthonormal under
    the real-space inner product, and the original deviations equal
    sum_j R_ji q_j with R upper triangular, exp(log R_ii) on its diagonal."""
    N, L, eps = 32, 20.0, 1e-3
    X0 = O.to_compact(O.project_field(W.uniform_field(3, N, 1.0), L))
    D = [O.to_compact(O.project_field(W.uniform_field(10 + i, N, 1.0), L)) for i in range(4)]
    D[2] = D[2] + 0.9 * D[0]  # not orthogonal to begin with
    logs, Xs = O.lyapunov_qr(X0, [X0 + eps * d for d in D], eps, N)
    q = [(X - X0) / eps for X in Xs]
    for i in range(4):
        for j in range(4):
            assert abs(O.lyap_inner(q[i], q[j], N) - (i == j)) < 1e-10
    for i in range(4):
        r = [O.lyap_inner(q[j], D[i], N) for j in range(4)]
        assert all(abs(r[j]) < 1e-8 * abs(r[i]) for j in range(i + 1, 4))  # triangular
        assert abs(math.log(r[i]) - logs[i]) < 1e-10
        rec = sum(r[j] * q[j] for j in range(i + 1))
        assert np.max(np.abs(rec - D[i])) < 1e-9 * np.max(np.abs(D[i]))


def test_lyapunov_linear_spectrum_closed_form():
    """With the nonlinear, advection and wall terms off, perturbations evolve
    by the exact multiplier exp(L(k) dt) per step, so the exponents are the
    largest values of L(k) = -alpha - Gamma0 k^2 - Gamma2 k^4 over the state
    space, each with its multiplicity: a shell of modes with one |m| gives
    two real directions per pair +-m (divergence-free velocity), k = 0 gives
    two (the mean flow).  Box L = 2 pi 1.2: shell |m| = 1 (k^2 = 1/1.44,
    4 directions) is the most unstable, then k = 0 (L = -alpha = 1, 2
    directions), then the shell |m|^2 = 2 (0.46)."""
    N, Lbox = 16, 2 * math.pi * 1.2
    p = dataclasses.replace(O.workload_params(dt=0.05), beta=0.0, lambda0=0.0, gamma_v=0.0, gamma_w=0.0)
    lam = lambda k2: -p.alpha - p.gamma0 * k2 - p.gamma2 * k2 * k2
    k1 = 1.0 / 1.44
    want = [lam(k1)] * 4 + [lam(0.0)] * 2
    assert lam(2 * k1) < lam(0.0) < lam(k1) and all(lam(m2 * k1) < lam(2 * k1) for m2 in (4, 5, 8, 9))
    # base: the zero state (a fixed point; with growth rates > 0 any other base
    # would grow by e^48 over the run and swamp eps-sized differences)
    v0 = np.zeros((2, N, N), dtype=np.complex128)
    perts = [O.project_field(W.uniform_field(20 + i, N, 1e-3), Lbox) for i in range(6)]
    tau = 20
    logs = O.lyapunov_run(v0, perts, np.zeros((N, N)), p, Lbox, 1e-6, tau, 60)
    got = logs[-1] / (tau * p.dt)
    assert np.max(np.abs(got - np.array(want))) < 1e-8, got
    # the time average converges to the same values (start-up transient / T)
    avg = logs.mean(axis=0) / (tau * p.dt)
    assert np.max(np.abs(avg - np.array(want))) < 0.05


# ---- temporal power spectral density of the vorticity --------------------------------------
def test_temporal_psd_closed_forms():
    """S(f) of eq. (PSD) for fields whose time sums are known: a pattern
    cos(k.x - 2 pi f0 t) sampled over whole periods gives (T/2)^2 at f = +-f0
    and 0 at the other multiples of 1/(T dt); a constant field c gives
    (c T)^2 at f = 0; S is even in f for real fields."""
    N, L, T, dt = 16, 10.0, 40, 0.5
    x, y = O.node_coords(N, L)
    f0 = 3 / (T * dt)  # three periods over the record
    times = np.arange(T) * dt
    k = 2 * np.pi / L * np.array([2.0, 1.0])
    series = [np.cos(k[0] * x + k[1] * y - 2 * np.pi * f0 * t) for t in times]
    freqs = np.array([j / (T * dt) for j in range(-5, 6)])
    S = O.temporal_psd(series, times, freqs)
    want = np.where(np.isclose(np.abs(freqs), f0), (T / 2) ** 2, 0.0)
    assert np.max(np.abs(S - want)) < 1e-9 * T * T
    S0 = O.temporal_psd([np.full((N, N), 0.7)] * T, times, [0.0, 1 / (T * dt)])
    assert abs(S0[0] - (0.7 * T) ** 2) < 1e-9 and abs(S0[1]) < 1e-9
    rng = np.random.default_rng(4)
    noise = [rng.standard_normal((N, N)) for _ in range(T)]
    fr = np.array([0.013, 0.21, 0.37])
    assert np.allclose(O.temporal_psd(noise, times, fr), O.temporal_psd(noise, times, -fr), rtol=1e-12)


# ---- pins added for the diagnostics, the Algorithm 2 cutoff and the paper preset ------------------
def test_norms_against_real_space_sums():
    """norms(): Parseval sum, mean and max |k . v_hat| against quantities fixed
    in real space.  A field made of a constant, a cosine along x in v_x only
    and a divergence-free mode: sum |v|^2 and the mean are plain sums over the
    nodes; the divergence d_x v_x = -A k sin(k x) has unitary spectrum of
    modulus A k N / 2 at m = (+-m0, 0), so max |k . v_hat| = A k N / 2."""
    N, L, A, m0 = 32, 20.0, 0.7, 3
    x, y = O.node_coords(N, L)
    k = 2 * math.pi * m0 / L
    v = 0.2 * mode_field(N, L, 2, 1)
    v[0] += 0.25 + A * np.cos(k * x)
    v[1] += -0.4
    vh = O.dft2(v)
    e, mx, my, div = O.norms(vh, L)
    assert abs(e - float(np.sum(v * v))) < 1e-12 * float(np.sum(v * v))
    assert abs(mx - float(v[0].mean())) < 1e-15 and abs(my - float(v[1].mean())) < 1e-15
    assert abs(mx - 0.25) < 1e-14 and abs(my + 0.4) < 1e-14
    assert abs(div - A * k * N / 2) < 1e-12 * A * k * N
    # a divergence-free field has no divergence left beyond rounding
    _, _, _, div0 = O.norms(O.dft2(mode_field(N, L, 2, 1)), L)
    assert div0 < 1e-13


def test_alg2_cutoff_keeps_the_edge_and_drops_beyond():
    """Algorithm 2 removes modes with k^2 > (pi/(4 dx))^2, i.e. m^2 > (N/8)^2
    (strict): a mode with m^2 = (N/8)^2 survives, one with m^2 = (N/8)^2 + 1
    does not.  With K_naive = c + a cos(edge) + b cos(beyond) the result is
    therefore (c + a cos(edge))^2 exactly, up to rounding."""
    N, L = 64, 64.0
    x, y = O.node_coords(N, L)
    g = 2 * math.pi / L
    edge = np.cos(g * (8 * x))              # m = (8, 0): m^2 = 64 = (N/8)^2, kept
    beyond = np.cos(g * (7 * x + 4 * y))    # m = (7, 4): m^2 = 65, removed
    c, a, b = 0.5, 0.3, 0.2
    K = O.mask_alg2(c + a * edge + b * beyond)
    assert np.abs(K - (c + a * edge) ** 2).max() < 1e-14


def test_paper_preset_is_table_one():
    """The paper preset against the literal values of the table of parameters
    (Appendix A): lambda = 9, a = 0.5, b = 1.6, gamma_v = 40, gamma_w = 4,
    dt = 0.01; eq. (2)'s linear part a v - (1 + lap)^2 v has the symbol
    a - (1 - k^2)^2."""
    lam, a, b, gv, gw, dt = 9.0, 0.5, 1.6, 40.0, 4.0, 0.01
    p = O.paper_params()
    assert (p.lambda0, p.beta, p.gamma_v, p.gamma_w, p.dt, p.lambda1) == (lam, b, gv, gw, dt, 0.0)
    k2 = np.array([0.0, 0.25, 1.0, 1.7, 4.0])
    assert np.abs(O.linear_symbol(k2, p) - (a - (1.0 - k2) ** 2)).max() < 1e-14


# ---- fourth-order exponential Runge-Kutta (ETDRK4, Cox and Matthews 2002) ---------------------
def test_phi_123_match_high_precision():
    """phi_k(z) = sum_j z^j/(j+k)!, k = 1, 2, 3, against 40-digit evaluations
    of their closed forms, across the series / recurrence switch at |z| = 1/2
    and into the stiff range."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    z = np.array([0.0, 1e-12, -3e-6, 4e-3, -0.3, 0.49, -0.5, 0.51, -2.0, 1.25, -80.0, -5e3])
    got = O.phi_123(z)
    for i, zi in enumerate(z):
        if zi == 0.0:
            want = (1.0, 0.5, 1.0 / 6.0)
        else:
            q = mpmath.mpf(float(zi))
            e = mpmath.expm1(q)
            want = (float(e / q), float((e - q) / q ** 2), float((e - q - q * q / 2) / q ** 3))
        for k in range(3):
            assert abs(got[k][i] - want[k]) <= 1e-13 * abs(want[k]), (zi, k, got[k][i], want[k])


def _etdrk4_scalar(z, w):
    """Amplification of ETDRK4 on u' = (L + lam) u with z = L h, w = lam h,
    worked out by hand from the scheme's four stages (phi functions from 40
    digits): a = (e^{z/2} + q w) u with q = phi_1(z/2)/2, b = e^{z/2} u + q w a,
    c = e^{z/2} a + q w (2 b - u), u' = e^z u + w (f1 u + 2 f2 (a + b) + f3 c)."""
    import mpmath
    mpmath.mp.dps = 40
    Z, Wm = mpmath.mpf(z), mpmath.mpf(w)
    ph = lambda k, x: sum(x ** j / mpmath.factorial(j + k) for j in range(60))
    E, E2, q = mpmath.exp(Z), mpmath.exp(Z / 2), ph(1, Z / 2) / 2
    f1 = ph(1, Z) - 3 * ph(2, Z) + 4 * ph(3, Z)
    f2 = ph(2, Z) - 2 * ph(3, Z)
    f3 = -ph(2, Z) + 4 * ph(3, Z)
    A = E2 + q * Wm
    B = E2 + q * Wm * A
    C = E2 * A + q * Wm * (2 * B - 1)
    return float(E + Wm * (f1 + 2 * f2 * (A + B) + f3 * C))


def test_etdrk4_linear_forcing_closed_form():
    """With a constant mask K = c and beta = lambda0 = 0 the forcing is the
    linear -gamma_v c v, so every mode follows u_n = R^n u_0 with R the
    scheme's scalar amplification (worked out by hand, above); and R^n tends
    to the exact e^{(L - gamma_v c) t} at fourth order in h.  A stage fed the
    wrong state or a swapped coefficient fails the first check."""
    pytest.importorskip("mpmath")
    N, L, c, n = 16, 2 * math.pi * 4.0, 0.3, 40
    p = dataclasses.replace(zero_nl(O.workload_params()), gamma_v=50.0, dt=0.02, scheme="etdrk4")
    v0 = O.project_field(mode_field(N, L, 1, 2) + mode_field(N, L, 3, 0, 0.5, 1.1), L)
    vh = O.run_velocity(v0, np.full((N, N), c), p, L, n)
    for mx, my in ((1, 2), (3, 0)):
        k2 = (2 * math.pi / L) ** 2 * (mx * mx + my * my)
        Lk = 1.0 + k2 - k2 * k2
        R = _etdrk4_scalar(Lk * p.dt, -p.gamma_v * c * p.dt)
        for comp in range(2):
            if abs(v0[comp, my % N, mx]) > 0:
                assert abs(vh[comp, my % N, mx] / v0[comp, my % N, mx] - R ** n) < 1e-12 * R ** n
    # the hand-worked amplification is a fourth-order approximation of the exponential
    Lk, lam, T = 1.0 + 0.5 - 0.25, -5.0, 0.4
    err = [abs(_etdrk4_scalar(Lk * h, lam * h) ** round(T / h) - math.exp((Lk + lam) * T)) for h in (0.02, 0.01, 0.005)]
    assert 15.0 < err[0] / err[1] < 18.0 and 15.0 < err[1] / err[2] < 17.5, err


@pytest.mark.parametrize("k2,rate", [(0.5, 1.25), (2.0, 1.0 + 2.0 - 4.0)])
def test_etdrk4_linear_modes_are_exact(k2, rate):
    """With the forcing switched off every stage reduces to the exponential:
    a single mode grows or decays at exactly L(k) (P3/P4)."""
    N, n = 16, 200
    p = dataclasses.replace(zero_nl(O.workload_params()), scheme="etdrk4")
    L = 2 * math.pi * math.sqrt(2.0 / k2)
    v0 = O.project_field(mode_field(N, L, 1, 1), L)
    vh = O.run_velocity(v0, np.zeros((N, N)), p, L, n)
    got = math.log(abs(vh[1, 1, 1]) / abs(v0[1, 1, 1])) / (n * p.dt)
    assert abs(got - rate) < 1e-11, (got, rate)


@pytest.mark.parametrize("preset", ["workload", "paper"])
def test_etdrk4_fourth_order_convergence(preset):
    """Errors against the finest run scale as dt^4: for dt = 8h, 4h, 2h against
    h the differences are c (8^4 - 1, 4^4 - 1, 2^4 - 1) h^4, ratios 273 and 17
    (a third-order slip gives 73 and 9).  The paper preset exercises the
    gamma_w source."""
    N, L = 16, 16.0
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v0 = O.project_field(W.uniform_field(11, N, 0.8), L)
    if preset == "workload":
        base, T_end, dts = dataclasses.replace(O.workload_params(), gamma_v=10.0), 0.4, (0.02, 0.01, 0.005, 0.0025)
    else:
        base, T_end, dts = dataclasses.replace(O.paper_params(), gamma_v=10.0, gamma_w=2.0), 0.2, (0.01, 0.005, 0.0025, 0.00125)
    out = {dt: O.run_velocity(v0, K, dataclasses.replace(base, dt=dt, scheme="etdrk4"), L, int(round(T_end / dt)))
           for dt in dts}
    e = [np.abs(out[dt] - out[dts[-1]]).max() for dt in dts[:3]]
    assert 240.0 < e[0] / e[2] < 330.0 and 16.0 < e[1] / e[2] < 19.0, e


def test_etdrk4_solves_the_same_equation_as_etdrk2():
    """ETDRK4 at dt and ETD2RK at dt/4 approach the same solution: their
    difference is below a tenth of ETD2RK's own change from dt to dt/4
    (ETD2RK's error shrinks 16-fold, ETDRK4's is far smaller)."""
    N, L, T_end, dt = 16, 16.0, 0.4, 0.01
    K = O.mask_tanh(N, L, [(0, 0)], [5.0], 0.5)
    v0 = O.project_field(W.uniform_field(11, N, 0.8), L)
    base = dataclasses.replace(O.workload_params(), gamma_v=10.0)
    e4 = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt, scheme="etdrk4"), L, int(round(T_end / dt)))
    e2a = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt, scheme="etdrk2"), L, int(round(T_end / dt)))
    e2b = O.run_velocity(v0, K, dataclasses.replace(base, dt=dt / 4, scheme="etdrk2"), L, int(round(4 * T_end / dt)))
    assert np.abs(e4 - e2b).max() < 0.1 * np.abs(e2a - e2b).max()


def test_etdrk4_stays_divergence_free_and_hermitian():
    N, L = 32, 32.0
    K = O.mask_tanh(N, L, [(0, 0)], [10.0], 0.5)
    p = dataclasses.replace(O.workload_params(), scheme="etdrk4")
    vh = O.project_field(W.uniform_field(13, N, 0.01), L)
    kx, ky, _, _ = O.grid(N, L)
    vh = O.run_velocity(vh, K, p, L, 600)
    assert np.abs(kx * vh[0] + ky * vh[1]).max() < 1e-13 * np.abs(vh).max()
    assert np.array_equal(vh, np.conj(O.reflect(vh)))
