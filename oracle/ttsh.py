"""FP64 CPU oracle of the damped TTSH time step (test infrastructure only).

What is computed follows the paper's method section (model eqs. (1)-(4),
computation and mask-generation subsections), Appendix C (Algorithm 1, the
integration scheme, and the text after it: unitary DFT, the exponential
multiplier, the k = 0 rule of eq. (7), the 1/2-rule cutoff, the Hermitian
correction, the stream function) and Appendix D (Algorithm 2, the automatic
mask generator).  The diagnostics follow the results sections: the order
parameters Psi (circle) and Psi_2 (dumbbell, its regions of radius D/2), the
temporal power spectral density of the vorticity (eq. (PSD)), a vortex count,
and Lyapunov exponents by perturbed copies and QR re-orthonormalisation.

General coefficient form.  The paper writes the model in the dimensionless
(a, b, lambda, gamma_v, gamma_w) convention, eq. (2)/(4).  The workloads used
here are quoted in the (alpha, beta, Gamma0, Gamma2, lambda0, lambda1)
convention of the Toner-Tu/Swift-Hohenberg literature the paper cites.  Both
are special cases of

    div v = 0,
    dv/dt + lambda0 (v.grad) v = -grad p + lambda1 grad|v|^2
                                 - (alpha + beta |v|^2) v
                                 + Gamma0 lap v - Gamma2 lap^2 v
                                 - gamma_v K v
    plus, in the vorticity equation, the extra damping  -gamma_w K omega,

whose linear Fourier symbol is  L(k) = -alpha - Gamma0 k^2 - Gamma2 k^4.
The paper's a - (1 - k^2)^2 is alpha = 1 - a, Gamma0 = -2, Gamma2 = 1.

Conventions: forward DFT carries e^{-ik.x}
and is unitary (1/N per 2D transform, Appendix C); a spatial derivative is the
multiplier +ik, which is what Algorithm 1 and the stream-function relations of
Appendix A use (the prose sentence after Algorithm 1 has the opposite sign,
taken as a slip).  Arrays are [component][y][x], component 0 = x; grid node
(i, j) sits at x = (j - N/2) dx, y = (i - N/2) dx.  Spectra are in FFT order,
axis -2 = m_y, axis -1 = m_x, k = (2 pi / L) m.

The dealiasing radius is M = N/4: a mode is removed when
m_x^2 + m_y^2 > M^2 (the 1/2 rule, k^2 > (pi/(2 dx))^2, strict inequality).
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np
import scipy.fft as sfft

_WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Params:
    """Coefficients of the general form above, plus the time step.

    scheme: 'ifeuler' (Algorithm 1: integrating factor + Euler, the default),
            'etd1'    (exponential Euler with phi_1 weighting of the forcing),
            'imex'    (linearly implicit Euler on the stiff operator),
            'etdrk2'  (second-order exponential Runge-Kutta, two forcing
                       evaluations per step; see velocity_step_etdrk2),
            'etdrk4'  (fourth-order exponential Runge-Kutta, four forcing
                       evaluations per step; see velocity_step_etdrk4).
    """
    alpha: float = -1.0
    beta: float = 1.0
    gamma0: float = -1.0
    gamma2: float = 1.0
    lambda0: float = 3.0
    lambda1: float = 0.0
    gamma_v: float = 100.0
    gamma_w: float = 0.0
    dt: float = 0.01
    scheme: str = "ifeuler"


def paper_params(dt: float = 0.01) -> Params:
    """The paper's preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)
    (model subsection; Table I), mapped to the general form."""
    a, b, lam = 0.5, 1.6, 9.0
    return Params(alpha=1.0 - a, beta=b, gamma0=-2.0, gamma2=1.0, lambda0=lam,
                  lambda1=0.0, gamma_v=40.0, gamma_w=4.0, dt=dt)


def workload_params(dt: float = 0.01) -> Params:
    """Gamma0 = -1, Gamma2 = 1, alpha = -1, beta = 1, lambda0 = 3, lambda1 = 0,
    one penalisation kappa = 100 taken as gamma_v, gamma_w = 0."""
    return Params(dt=dt)


# ---------------------------------------------------------------------------
# grid and transforms
# ---------------------------------------------------------------------------
def mode_index(N: int) -> np.ndarray:
    """Integer mode numbers in FFT order: 0, 1, ..., N/2-1, -N/2, ..., -1."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)


def grid(N: int, L: float):
    """Return (kx, ky, k2, m2) on the full N x N spectrum in FFT order
    (Table I: k in [-pi/dx, pi/dx]^2, spacing 2 pi / L)."""
    m = mode_index(N)
    dk = 2.0 * math.pi / L
    mx = m[None, :]
    my = m[:, None]
    kx = dk * mx * np.ones((N, 1))
    ky = dk * my * np.ones((1, N))
    m2 = mx * mx + my * my
    k2 = kx * kx + ky * ky
    return kx, ky, k2, m2


def dft2(f: np.ndarray) -> np.ndarray:
    """Unitary forward DFT over the last two axes (Appendix C definition)."""
    return sfft.fft2(f, axes=(-2, -1), norm="ortho", workers=_WORKERS)


def idft2(F: np.ndarray) -> np.ndarray:
    """Unitary inverse DFT over the last two axes (Appendix C definition)."""
    return sfft.ifft2(F, axes=(-2, -1), norm="ortho", workers=_WORKERS)


def dft2_bruteforce(f: np.ndarray, sign: int = -1) -> np.ndarray:
    """The Appendix C definition summed term by term, O(N^4): tiny N only.

    sign = -1 is the forward DFT, +1 the inverse; both carry 1/sqrt(N^2).
    """
    f = np.asarray(f, dtype=np.complex128)
    N = f.shape[-1]
    assert f.shape[-2] == N and N <= 32
    out = np.zeros_like(f)
    idx = np.arange(N)
    for my in range(N):
        for mx in range(N):
            phase = np.exp(sign * 2j * math.pi * (my * idx[:, None] + mx * idx[None, :]) / N)
            out[..., my, mx] = (f * phase).sum(axis=(-2, -1)) / N
    return out


def reflect(F: np.ndarray) -> np.ndarray:
    """F(-k) in FFT order: index m -> (-m) mod N on both spectral axes."""
    return np.roll(np.flip(F, axis=(-2, -1)), 1, axis=(-2, -1))


# ---------------------------------------------------------------------------
# linear operator
# ---------------------------------------------------------------------------
def linear_symbol(k2: np.ndarray, p: Params) -> np.ndarray:
    """L(k) = -alpha - Gamma0 k^2 - Gamma2 k^4 (general form; the paper's
    a - (1 - k^2)^2 of Algorithm 1 is the special case)."""
    return -p.alpha - p.gamma0 * k2 - p.gamma2 * k2 * k2


def linear_factors(k2: np.ndarray, p: Params):
    """Weights (A, B) of the one-step map  u' = A u + B dt f  for the stiff
    linear part.

    ifeuler: A = B = exp(L dt)            (Algorithm 1, exponential multiplier)
    etd1:    A = exp(L dt), B = (exp(L dt) - 1)/(L dt)   (B = 1 at L = 0)
    imex:    A = B = 1/(1 - L dt)
    """
    z = linear_symbol(k2, p) * p.dt
    if p.scheme == "ifeuler":
        E = np.exp(z)
        return E, E
    if p.scheme == "etd1":
        E = np.exp(z)
        with np.errstate(divide="ignore", invalid="ignore"):
            phi = np.where(z == 0.0, 1.0, np.expm1(z) / np.where(z == 0.0, 1.0, z))
        return E, phi
    if p.scheme == "imex":
        A = 1.0 / (1.0 - z)
        return A, A
    raise ValueError(p.scheme)


def phi_functions(z: np.ndarray):
    """phi_1(z) = (e^z - 1)/z and phi_2(z) = (e^z - 1 - z)/z^2 (both at z = 0 by
    continuity, 1 and 1/2), from expm1; for |z| < 1e-2 phi_2 by its Taylor
    series sum_j z^j/(j+2)!, which avoids the cancellation in e^z - 1 - z."""
    z = np.asarray(z, dtype=np.float64)
    small = np.abs(z) < 1e-2
    zs = np.where(small, 1.0, z)
    em1 = np.expm1(z)
    phi1 = np.where(z == 0.0, 1.0, em1 / np.where(z == 0.0, 1.0, z))
    series = sum(z ** j / math.factorial(j + 2) for j in range(7))
    phi2 = np.where(small, series, (em1 - z) / (zs * zs))
    return phi1, phi2


# ---------------------------------------------------------------------------
# projections
# ---------------------------------------------------------------------------
def dealias_keep(N: int) -> np.ndarray:
    """True where a mode survives the 1/2 rule: m_x^2 + m_y^2 <= (N/4)^2."""
    _, _, _, m2 = grid(N, 1.0)
    M = N // 4
    return m2 <= M * M


def hermitian_fix(F: np.ndarray) -> np.ndarray:
    """F(k) <- (F(k) + F(-k)^*)/2 (Algorithm 1, Hermitian correction of the
    surviving modes; Appendix C says it is essential for stability)."""
    return 0.5 * (F + np.conj(reflect(F)))


def leray(vhat: np.ndarray, kx: np.ndarray, ky: np.ndarray, k2: np.ndarray) -> np.ndarray:
    """Divergence-free part, P(k) = I - k k^T / k^2, for k != 0; k = 0 kept."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    div = kx * vhat[0] + ky * vhat[1]
    return np.stack([vhat[0] - kx * div * inv, vhat[1] - ky * div * inv])


def project_field(v0: np.ndarray, L: float) -> np.ndarray:
    """Initial projection of an arbitrary real field onto the state space of
    the scheme: DFT, 1/2-rule cutoff, Leray (k != 0), Hermitian fix.  Returns
    the full unitary spectrum v_hat [2][N][N]."""
    N = v0.shape[-1]
    kx, ky, k2, _ = grid(N, L)
    vh = dft2(np.asarray(v0, dtype=np.float64))
    vh = vh * dealias_keep(N)
    vh = leray(vh, kx, ky, k2)
    return hermitian_fix(vh)


def vorticity_hat(vhat: np.ndarray, kx: np.ndarray, ky: np.ndarray) -> np.ndarray:
    """omega_hat = i (k_x v_y - k_y v_x) (omega = d_x v_y - d_y v_x, model subsection)."""
    return 1j * (kx * vhat[1] - ky * vhat[0])


def velocity_from_vorticity(w_hat: np.ndarray, kx, ky, k2) -> np.ndarray:
    """Stream function psi_hat = omega_hat / k^2, v = (i k_y psi, -i k_x psi)
    (Algorithm 1, stream-function step; Appendix A: lap psi = -omega, v_x = d_y psi,
    v_y = -d_x psi).  The k = 0 entry is returned as 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        psi = np.where(k2 > 0, w_hat / np.where(k2 > 0, k2, 1.0), 0.0)
    return np.stack([1j * ky * psi, -1j * kx * psi])


# ---------------------------------------------------------------------------
# Algorithm 1, as printed (vorticity form, convective advection)
# ---------------------------------------------------------------------------
def alg1_init(v0: np.ndarray, L: float):
    """Consistent Algorithm 1 state (v, omega_hat) from an arbitrary field."""
    N = v0.shape[-1]
    kx, ky, _, _ = grid(N, L)
    vh = project_field(v0, L)
    return idft2(vh).real, vorticity_hat(vh, kx, ky)


def alg1_step(v: np.ndarray, w_hat: np.ndarray, K: np.ndarray, p: Params, L: float):
    """One step of Algorithm 1 in the general coefficient form.

    REQUIRE (v(t), omega_hat(t)); ENSURE (v(t+dt), omega_hat(t+dt)).
    """
    N = v.shape[-1]
    M = N // 4
    kx, ky, k2, m2 = grid(N, L)
    vx, vy = v[0], v[1]
    # real-space forcing: rhs_1 = -b |v|^2 v - gamma_v K v
    vsq = vx * vx + vy * vy
    rhs1 = np.stack([-p.beta * vsq * vx - p.gamma_v * K * vx,
                     -p.beta * vsq * vy - p.gamma_v * K * vy])
    # convective term: rhs_2 = -lambda v . iDFT[i k omega_hat] - gamma_w K omega
    w = idft2(w_hat).real
    dwx = idft2(1j * kx * w_hat).real
    dwy = idft2(1j * ky * w_hat).real
    rhs2 = -p.lambda0 * (vx * dwx + vy * dwy) - p.gamma_w * K * w
    # curl in k-space: rhs_hat = i k x DFT[rhs_1] + DFT[rhs_2]
    r1 = dft2(rhs1)
    rhs_hat = 1j * (kx * r1[1] - ky * r1[0]) + dft2(rhs2)
    # Euler step with exponential multiplier: exp(L dt)(omega_hat + dt rhs_hat)
    A, B = linear_factors(k2, p)
    w_naive = A * w_hat + B * p.dt * rhs_hat
    # per-k post-processing
    w_new = hermitian_fix(w_naive)                       # Hermitian correction
    cut = m2 > M * M
    w_new[cut] = 0.0                                     # 1/2-rule cutoff
    w_new[0, 0] = 0.0                                    # omega_hat(0) = 0
    vh_new = velocity_from_vorticity(w_new, kx, ky, k2)  # stream function; cut modes stay 0
    # mean flow from the averaged equation (7): exp(L(0) dt) DFT[v + dt rhs_1](0)
    A0, B0 = A[0, 0], B[0, 0]
    vh0 = dft2(v)[:, 0, 0]
    vh_new[:, 0, 0] = A0 * vh0 + B0 * p.dt * r1[:, 0, 0]
    v_new = idft2(vh_new).real
    return v_new, w_new


# ---------------------------------------------------------------------------
# velocity / Leray form (independent formulation, the one the GPU evolves)
# ---------------------------------------------------------------------------
def velocity_rhs(vhat: np.ndarray, K: np.ndarray, p: Params, L: float):
    """Real-space forcing of the velocity form, transformed.

    Uses (v.grad) v = grad(|v|^2/2) + omega v_perp, v_perp = (-v_y, v_x); the
    gradient part (and lambda1 grad|v|^2) is removed by the projection, but it
    is kept here so that the test of its removal is meaningful.

    Returns (N_hat, rhs1_hat, G_hat): the full forcing, the part from
    -beta|v|^2 v - gamma_v K v alone (what the k = 0 rule uses) and the
    vorticity source -gamma_w K omega.
    """
    N = vhat.shape[-1]
    kx, ky, _, _ = grid(N, L)
    v = idft2(vhat).real
    w_hat = vorticity_hat(vhat, kx, ky)
    w = idft2(w_hat).real
    vx, vy = v[0], v[1]
    vsq = vx * vx + vy * vy
    rhs1 = np.stack([-(p.beta * vsq + p.gamma_v * K) * vx,
                     -(p.beta * vsq + p.gamma_v * K) * vy])
    adv = -p.lambda0 * np.stack([w * (-vy), w * vx])
    grad_half = -p.lambda0 * 0.5 * vsq          # -lambda0 grad(|v|^2/2)
    r1 = dft2(rhs1)
    gh = dft2(grad_half + p.lambda1 * vsq)
    N_hat = r1 + dft2(adv) + np.stack([1j * kx * gh, 1j * ky * gh])
    G_hat = dft2(-p.gamma_w * K * w)
    return N_hat, r1, G_hat


def velocity_step(vhat: np.ndarray, K: np.ndarray, p: Params, L: float) -> np.ndarray:
    """One step on the spectral velocity v_hat (full unitary spectrum).

    v_hat' = P(k)[A v_hat + B dt N_hat] + B dt (i k_y, -i k_x) G_hat / k^2
    for 0 < m^2 <= M^2;  v_hat'(0) = A(0) v_hat(0) + B(0) dt rhs1_hat(0);
    0 for m^2 > M^2;  then the Hermitian correction.  Its curl is Algorithm 1's
    omega update (identical up to rounding), which the tests check.

    The projection acts on the whole update, not on the forcing alone:
    Algorithm 1 rebuilds v from the stream function of the new omega every
    step, so v is divergence-free after every step.  Projecting only the
    forcing would leave the rounding error's divergent part to be multiplied
    by e^{L dt} each step, which grows wherever L(k) > 0.
    """
    N = vhat.shape[-1]
    M = N // 4
    kx, ky, k2, m2 = grid(N, L)
    N_hat, r1, G_hat = velocity_rhs(vhat, K, p, L)
    A, B = linear_factors(k2, p)
    out = leray(A * vhat + B * p.dt * N_hat, kx, ky, k2) \
        + B * p.dt * velocity_from_vorticity(G_hat, kx, ky, k2)
    out[:, 0, 0] = A[0, 0] * vhat[:, 0, 0] + B[0, 0] * p.dt * r1[:, 0, 0]
    out = out * (m2 <= M * M)
    return hermitian_fix(out)


def velocity_step_etdrk2(vhat: np.ndarray, K: np.ndarray, p: Params, L: float) -> np.ndarray:
    """One step of the second-order exponential Runge-Kutta scheme (Cox and
    Matthews, J. Comput. Phys. 176 (2002), the ETD2RK scheme) on the same
    velocity form, z = L(k) dt:

        a   = e^z u + dt phi_1(z) F(u)
        u'  = a + dt phi_2(z) (F(a) - F(u))

    where F is the forcing of velocity_step, acting through the same rules:
    the projection P(k) of the whole update and the lifted vorticity source
    for 0 < m^2 <= M^2, only the rhs1 part at k = 0, zero beyond the 1/2 rule,
    then the Hermitian correction (after each stage).  Exact for the linear
    part, second order in dt overall.
    """
    N = vhat.shape[-1]
    M = N // 4
    kx, ky, k2, m2 = grid(N, L)
    E = np.exp(linear_symbol(k2, p) * p.dt)
    phi1, phi2 = phi_functions(linear_symbol(k2, p) * p.dt)
    keep = m2 <= M * M

    def stage(base, wbase, f, r1, g, w):
        out = leray(wbase * base + w * p.dt * f, kx, ky, k2) + w * p.dt * velocity_from_vorticity(g, kx, ky, k2)
        out[:, 0, 0] = wbase[0, 0] * base[:, 0, 0] + w[0, 0] * p.dt * r1[:, 0, 0]
        return hermitian_fix(out * keep)

    Fu, r1u, Gu = velocity_rhs(vhat, K, p, L)
    a = stage(vhat, E, Fu, r1u, Gu, phi1)
    Fa, r1a, Ga = velocity_rhs(a, K, p, L)
    return stage(a, np.ones_like(E), Fa - Fu, r1a - r1u, Ga - Gu, phi2)


def phi_123(z: np.ndarray):
    """phi_1, phi_2, phi_3 with phi_k(z) = sum_j z^j/(j+k)!  (phi_0 = e^z,
    phi_k(z) = (phi_{k-1}(z) - 1/(k-1)!)/z).  For |z| < 1/2 the series (20
    terms) is summed; elsewhere phi_1 = expm1(z)/z and the recurrence, whose
    subtractions then lose at most a few bits."""
    z = np.asarray(z, dtype=np.float64)
    small = np.abs(z) < 0.5
    zs = np.where(small, 1.0, z)
    p1 = np.expm1(zs) / zs
    p2 = (p1 - 1.0) / zs
    p3 = (p2 - 0.5) / zs
    ser = [sum(z ** j / math.factorial(j + k) for j in range(20)) for k in (1, 2, 3)]
    return np.where(small, ser[0], p1), np.where(small, ser[1], p2), np.where(small, ser[2], p3)


def velocity_step_etdrk4(vhat: np.ndarray, K: np.ndarray, p: Params, L: float) -> np.ndarray:
    """One step of the fourth-order exponential Runge-Kutta scheme of Cox and
    Matthews (J. Comput. Phys. 176 (2002), ETDRK4) on the velocity form, with
    h = dt and z = L(k) h:

        a  = e^{z/2} u + (h/2) phi_1(z/2) F(u)
        b  = e^{z/2} u + (h/2) phi_1(z/2) F(a)
        c  = e^{z/2} a + (h/2) phi_1(z/2) (2 F(b) - F(u))
        u' = e^z u + h [f1 F(u) + 2 f2 (F(a) + F(b)) + f3 F(c)]

    with f1 = phi_1 - 3 phi_2 + 4 phi_3, f2 = phi_2 - 2 phi_3 and
    f3 = -phi_2 + 4 phi_3 at z (the scheme's coefficients
    [-4 - z + e^z (4 - 3z + z^2)]/z^3, [2 + z + e^z (z - 2)]/z^3 and
    [-4 - 3z - z^2 + e^z (4 - z)]/z^3 written through the phi functions).
    Every stage applies Algorithm 1's rules as the other schemes do: the
    projection P(k) of the whole update and the lifted vorticity source for
    0 < m^2 <= M^2, only the rhs1 part of the forcing at k = 0, zero beyond
    the 1/2 rule, then the Hermitian correction.  Exact for the linear part,
    fourth order in h overall."""
    N = vhat.shape[-1]
    M = N // 4
    kx, ky, k2, m2 = grid(N, L)
    h = p.dt
    z = linear_symbol(k2, p) * h
    E, E2 = np.exp(z), np.exp(z / 2)
    Q = 0.5 * h * phi_123(z / 2)[0]
    p1, p2, p3 = phi_123(z)
    f1, f2, f3 = p1 - 3.0 * p2 + 4.0 * p3, p2 - 2.0 * p3, -p2 + 4.0 * p3
    keep = m2 <= M * M

    def stage(base, wbase, f, r1, g):
        """P(wbase base + f) + lift(g) for k != 0, wbase base + r1 at k = 0
        (f, r1, g already weighted)."""
        out = leray(wbase * base + f, kx, ky, k2) + velocity_from_vorticity(g, kx, ky, k2)
        out[:, 0, 0] = wbase[0, 0] * base[:, 0, 0] + r1[:, 0, 0]
        return hermitian_fix(out * keep)

    Fu, Ru, Gu = velocity_rhs(vhat, K, p, L)
    a = stage(vhat, E2, Q * Fu, Q * Ru, Q * Gu)
    Fa, Ra, Ga = velocity_rhs(a, K, p, L)
    b = stage(vhat, E2, Q * Fa, Q * Ra, Q * Ga)
    Fb, Rb, Gb = velocity_rhs(b, K, p, L)
    c = stage(a, E2, Q * (2 * Fb - Fu), Q * (2 * Rb - Ru), Q * (2 * Gb - Gu))
    Fc, Rc, Gc = velocity_rhs(c, K, p, L)

    def comb(xu, xa, xb, xc):
        return h * (f1 * xu + 2.0 * f2 * (xa + xb) + f3 * xc)

    return stage(vhat, E, comb(Fu, Fa, Fb, Fc), comb(Ru, Ra, Rb, Rc), comb(Gu, Ga, Gb, Gc))


def run_velocity(vhat: np.ndarray, K: np.ndarray, p: Params, L: float, nsteps: int) -> np.ndarray:
    step = {"etdrk2": velocity_step_etdrk2, "etdrk4": velocity_step_etdrk4}.get(p.scheme, velocity_step)
    for _ in range(nsteps):
        vhat = step(vhat, K, p, L)
    return vhat


def field(vhat: np.ndarray) -> np.ndarray:
    """Real velocity field from its unitary spectrum."""
    return idft2(vhat).real


def resample(vhat: np.ndarray, N_dst: int) -> np.ndarray:
    """Continuation between runs on different grids (the circle section's
    hysteresis protocol seeds each run from the previous final state): copy
    the spectrum by integer mode index, keeping the modes inside both grids'
    1/2-rule disks.  With the box side scaled with R, mode m is the same
    physical pattern on both grids; the unitary DFT carries a factor N, hence
    the scale N_dst/N_src."""
    N_src = vhat.shape[-1]
    Ms, Md = N_src // 4, N_dst // 4
    lim = min(Ms, Md) ** 2
    out = np.zeros(vhat.shape[:-2] + (N_dst, N_dst), dtype=np.complex128)
    for my in range(-min(Ms, Md), min(Ms, Md) + 1):
        for mx in range(-min(Ms, Md), min(Ms, Md) + 1):
            if mx * mx + my * my <= lim:
                out[..., my % N_dst, mx % N_dst] = vhat[..., my % N_src, mx % N_src] * (N_dst / N_src)
    return out


# ---------------------------------------------------------------------------
# masks (method section "mask generation"; Appendix D)
# ---------------------------------------------------------------------------
def node_coords(N: int, L: float):
    """Physical coordinates (x, y) of the nodes: x = (j - N/2) dx, y = (i - N/2) dx."""
    dx = L / N
    c = (np.arange(N, dtype=np.float64) - N / 2) * dx
    return c[None, :] * np.ones((N, 1)), c[:, None] * np.ones((1, N))


def mask_tanh(N: int, L: float, centers, radii, xi: float) -> np.ndarray:
    """Smoothed wall K = 1/2 [1 + tanh((r - R)/xi)] for one circle; for several
    circles the product of their outsides (the smooth AND of the outsides)."""
    x, y = node_coords(N, L)
    K = np.ones((N, N))
    for (cx, cy), R in zip(centers, radii):
        r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
        K = K * (0.5 * (1.0 + np.tanh((r - R) / xi)))
    return K


def mask_alg2(K_naive: np.ndarray) -> np.ndarray:
    """Algorithm 2: DFT of the binary mask, zero every mode with
    k^2 > (pi/(4 dx))^2 (m_x^2 + m_y^2 > (N/8)^2), inverse DFT, square.
    No optional modification.  The real part is taken before squaring."""
    N = K_naive.shape[-1]
    _, _, _, m2 = grid(N, 1.0)
    Kh = dft2(np.asarray(K_naive, dtype=np.float64))
    Kh[m2 > (N // 8) ** 2] = 0.0
    return idft2(Kh).real ** 2


# ---------------------------------------------------------------------------
# compact half spectrum (the library's state layout, for comparisons)
# ---------------------------------------------------------------------------
def to_compact(vhat: np.ndarray) -> np.ndarray:
    """Full FFT-order spectrum [..., N, N] -> compact [..., 2M+1, M+1] holding
    m_y = -M..M (row m_y + M) and m_x = 0..M."""
    N = vhat.shape[-1]
    M = N // 4
    rows = np.arange(-M, M + 1) % N
    return vhat[..., rows, :][..., : M + 1]


def from_compact(c: np.ndarray, N: int) -> np.ndarray:
    """Inverse of to_compact, filling m_x < 0 by Hermitian symmetry."""
    M = N // 4
    shape = c.shape[:-2] + (N, N)
    out = np.zeros(shape, dtype=np.complex128)
    my = np.arange(-M, M + 1)
    for mx in range(M + 1):
        out[..., my % N, mx] = c[..., :, mx]
        if mx > 0:
            out[..., (-my) % N, (-mx) % N] = np.conj(c[..., :, mx])
    return out


# ---------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------
def norms(vhat: np.ndarray, L: float):
    """(sum_x |v|^2, <v_x>, <v_y>, max |k . v_hat|) in FP64 (Parseval for the first)."""
    N = vhat.shape[-1]
    kx, ky, _, _ = grid(N, L)
    e = float(np.sum(np.abs(vhat) ** 2))
    mean = vhat[:, 0, 0].real / N
    div = float(np.max(np.abs(kx * vhat[0] + ky * vhat[1])))
    return e, float(mean[0]), float(mean[1]), div


def vortex_order(v: np.ndarray, L: float, center=(0.0, 0.0)) -> float:
    """Vortex order parameter Psi (circle section, transition subsection):
    [sum |e_theta . v| / sum |v| - 2/pi] / (1 - 2/pi)."""
    N = v.shape[-1]
    x, y = node_coords(N, L)
    x = x - center[0]
    y = y - center[1]
    r = np.sqrt(x * x + y * y)
    with np.errstate(divide="ignore", invalid="ignore"):
        etx = np.where(r > 0, -y / np.where(r > 0, r, 1.0), 0.0)
        ety = np.where(r > 0, x / np.where(r > 0, r, 1.0), 0.0)
    num = np.sum(np.abs(etx * v[0] + ety * v[1]))
    den = np.sum(np.sqrt(v[0] ** 2 + v[1] ** 2))
    return float((num / den - 2.0 / math.pi) / (1.0 - 2.0 / math.pi))


def vortex_order2(w: np.ndarray, L: float, split_x: float = 0.0, D: float = 0.0, center_y: float = 0.0) -> float:
    """Order parameter Psi_2 of the two-chamber (dumbbell) section: with
    x_left / x_right the nodes of largest |omega| in the left and right
    regions, |w(x_left) + w(x_right)| / (|w(x_left)| + |w(x_right)|); 1 for
    co-rotating (ferromagnetic), 0 for counter-rotating vortices.  Regions:
    with D > 0 the paper's, the nodes within D/2 of either cavity centre
    (split_x -+ D/2, center_y), the node where the two disks touch going to
    the right one; with D = 0 the half-planes left of x = split_x and at or
    right of it.  Ties go to the first node in row-major order; NaN when a
    region holds no node."""
    N = w.shape[-1]
    x, y = node_coords(N, L)
    left = x < split_x
    right = ~left
    if D > 0:
        r2 = (0.5 * D) ** 2
        left = left & ((x - (split_x - 0.5 * D)) ** 2 + (y - center_y) ** 2 <= r2)
        right = right & ((x - (split_x + 0.5 * D)) ** 2 + (y - center_y) ** 2 <= r2)
    if not left.any() or not right.any():
        return float("nan")
    aw = np.abs(w)
    iL = int(np.argmax(np.where(left, aw, -1.0)))
    iR = int(np.argmax(np.where(right, aw, -1.0)))
    wl, wr = w.flat[iL], w.flat[iR]
    return float(abs(wl + wr) / (abs(wl) + abs(wr)))


def vortex_count(v: np.ndarray, K: np.ndarray, kmax: float, vmin: float):
    """Topological defects of the velocity direction field.  A node is inside
    when K < kmax and has a direction when |v| > vmin.  For every grid cell
    (nodes (i, j), (i, j+1), (i+1, j+1), (i+1, j), periodic, taken
    counter-clockwise) whose four corners are inside with a direction, the
    winding number n = (1/2 pi) sum of the corner-to-corner changes of the
    angle of v, each wrapped into (-pi, pi]; for every inside node without a
    direction (a defect sitting exactly on a node, as at the centre of a
    symmetric vortex) whose eight neighbours are inside with a direction, the
    same sum around that ring.  Vortex centres (of either sense of rotation)
    carry n = +1, saddles (hyperbolic stagnation points) n = -1.  Returns
    (sum of n where n > 0, sum of |n| where n < 0)."""
    th = np.arctan2(v[1], v[0])
    sp = np.hypot(v[0], v[1])
    inside = K < kmax
    good = inside & (sp > vmin)

    def winding(path):
        w = np.zeros(th.shape)
        for q in range(len(path)):
            a, b = path[q], path[(q + 1) % len(path)]
            d = np.roll(th, (-b[0], -b[1]), (0, 1)) - np.roll(th, (-a[0], -a[1]), (0, 1))
            w += d - 2 * np.pi * np.ceil((d - np.pi) / (2 * np.pi))  # into (-pi, pi]
        ok = np.ones(th.shape, dtype=bool)
        for a in path:
            ok &= np.roll(good, (-a[0], -a[1]), (0, 1))
        return np.rint(w / (2 * np.pi)).astype(np.int64) * ok

    cells = winding([(0, 0), (0, 1), (1, 1), (1, 0)])
    ring = winding([(-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1), (1, 0), (1, -1), (0, -1)])
    ring = ring * (inside & ~(sp > vmin))
    n = np.concatenate([cells.ravel(), ring.ravel()])
    return int(n[n > 0].sum()), int(-n[n < 0].sum())


def temporal_psd(w_series, times, freqs) -> np.ndarray:
    """Temporal power spectral density of the vorticity (circle section,
    eq. (PSD)): S(f) = (1/N^2) sum_x |sum_t w(x, t) e^{-2 pi i f t}|^2 over
    the sampled times t (frequency f in cycles per unit time, Omega = 2 pi f).
    w_series: sequence of real [N][N] vorticity fields, one per time."""
    w = np.asarray(w_series, dtype=np.float64)
    N = w.shape[-1]
    t = np.asarray(times, dtype=np.float64)
    out = np.zeros(len(freqs))
    for j, f in enumerate(freqs):
        A = np.tensordot(np.exp(-2j * np.pi * f * t), w, axes=(0, 0))
        out[j] = float(np.sum(np.abs(A) ** 2)) / (N * N)
    return out


# ---------------------------------------------------------------------------
# Lyapunov exponents (Benettin / Shimada-Nagashima method, circle section's
# characterisation of the transition): perturbed copies of the state are
# advanced with the same step and re-orthonormalised by a QR decomposition.
# ---------------------------------------------------------------------------
def compact_weights(N: int) -> np.ndarray:
    """Weights of the compact half spectrum [2M+1][M+1] under which the
    weighted sum of |c|^2 is the full-spectrum sum (1 on the m_x = 0 column,
    which holds both signs of m_y; 2 on m_x > 0, whose mirror images -m are
    not stored)."""
    M = N // 4
    w = np.full((2 * M + 1, M + 1), 2.0)
    w[:, 0] = 1.0
    return w


def lyap_inner(a: np.ndarray, b: np.ndarray, N: int) -> float:
    """<a, b> of two compact states [2][2M+1][M+1]: sum over components and
    stored modes of w Re(conj(a) b) — the L2 inner product of the real fields
    over the grid nodes (Parseval, unitary DFT)."""
    return float(np.sum(compact_weights(N)[None] * (np.conj(a) * b).real))


def lyapunov_qr(base: np.ndarray, perts, eps: float, N: int):
    """One re-orthonormalisation.  The deviations d_i = (X_i - X_0)/eps of
    the perturbed states from the base state are factored as D = Q R (Q
    orthonormal under lyap_inner, diag R > 0); returns (log R_ii, the new
    states X_0 + eps Q_i).  The factorisation is numpy's Householder QR in the
    coordinates sqrt(w) (Re, Im) of every stored entry."""
    sw = np.sqrt(compact_weights(N))[None]
    cols = [np.concatenate([((X - base) / eps * sw).real.ravel(), ((X - base) / eps * sw).imag.ravel()])
            for X in perts]
    Q, R = np.linalg.qr(np.stack(cols, axis=1))
    sign = np.sign(np.diag(R))
    Q = Q * sign[None]
    r = np.abs(np.diag(R))
    n = base.size
    out = []
    for i in range(len(perts)):
        q = (Q[:n, i] + 1j * Q[n:, i]).reshape(base.shape) / sw
        out.append(base + eps * q)
    return np.log(r), out


def lyapunov_run(vhat0: np.ndarray, perts0, K: np.ndarray, p: Params, L: float, eps: float, tau: int,
                 intervals: int):
    """Benettin's method on full spectra: the base state and the perturbed
    states are each advanced tau steps with velocity_step (or the chosen
    scheme), then lyapunov_qr on their compact forms; returns the per-interval
    log R_ii, shape [intervals][p] (the exponents are their time averages
    divided by tau * dt).  The perturbed states start from perts0 and are
    first orthonormalised about vhat0."""
    N = vhat0.shape[-1]
    X0 = to_compact(vhat0)
    _, Xs = lyapunov_qr(X0, [to_compact(q) for q in perts0], eps, N)
    vb = from_compact(X0, N)
    vs = [from_compact(X, N) for X in Xs]
    logs = []
    for _ in range(intervals):
        vb = run_velocity(vb, K, p, L, tau)
        vs = [run_velocity(v, K, p, L, tau) for v in vs]
        lr, Xs = lyapunov_qr(to_compact(vb), [to_compact(v) for v in vs], eps, N)
        logs.append(lr)
        vs = [from_compact(X, N) for X in Xs]
    return np.array(logs)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 over all entries, FP64 sums."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b * b)))


# ---------------------------------------------------------------------------
# D4 actions on a vector field about the node (N/2, N/2)
# ---------------------------------------------------------------------------
def rotate90(v: np.ndarray) -> np.ndarray:
    """Counter-clockwise quarter turn about the centre node, acting on a vector
    field [2][y][x]: v'(x) = R v(R^-1 x), R (a, b) = (-b, a)."""
    N = v.shape[-1]
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    # destination node (i', j') takes the source node ((N - j') mod N, i')
    src_i, src_j = (N - J) % N, I
    vx = v[0][src_i, src_j]
    vy = v[1][src_i, src_j]
    return np.stack([-vy, vx])


def reflect_x(v: np.ndarray) -> np.ndarray:
    """Mirror x -> -x about the centre node: v'(x, y) = (-v_x, v_y)(-x, y)."""
    N = v.shape[-1]
    j = (N - np.arange(N)) % N
    return np.stack([-v[0][:, j], v[1][:, j]])


def transpose_xy(v: np.ndarray) -> np.ndarray:
    """Mirror about the diagonal x <-> y: v'(x, y) = (v_y, v_x)(y, x)."""
    return np.stack([v[1].T, v[0].T])
