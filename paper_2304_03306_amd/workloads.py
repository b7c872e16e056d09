"""Seeded synthetic inputs and workload definitions.

This module holds no arithmetic of the method: it draws the random initial
fields and the reseed noise, lists the geometries (grid size N, box side L,
circle centres and radii, mask width) of each workload, and builds the binary
"where to mask" fields that Algorithm 2 takes as input.  Both the GPU path and
the CPU oracle receive their inputs from here, so that they start from the
same numbers.

Random numbers: numpy's PCG64 generator seeded with the stated integer, one
i.i.d. uniform draw per node and component, in FP64; a run in FP32 rounds the
field to FP32 before either side sees it.  The continuation noise that the
library draws on the device comes from the counter-based Philox-4x32-10
generator (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11); `philox4x32_10` below implements the same published
definition in Python, so that the oracle side sees the same numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np


def uniform_field(seed: int, N: int, amp: float = 0.01, precision: int = 64) -> np.ndarray:
    """i.i.d. U[-amp, amp] per node and component, shape [2][N][N] (component
    0 = x), rounded to the run precision and returned as float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.uniform(-amp, amp, size=(2, N, N))
    if precision == 32:
        v = v.astype(np.float32).astype(np.float64)
    return v


def binary_outside(N: int, L: float, centers, radii) -> np.ndarray:
    """Binary wall field for a union of disks: 1 where a node lies outside
    every disk (||x - c|| >= R for all circles), else 0; uint8 [N][N].
    Node (i, j) sits at x = (j - N/2) L/N, y = (i - N/2) L/N."""
    dx = L / N
    c = (np.arange(N, dtype=np.float64) - N / 2) * dx
    x = c[None, :]
    y = c[:, None]
    out = np.ones((N, N), dtype=bool)
    for (cx, cy), R in zip(centers, radii):
        out &= np.sqrt((x - cx) ** 2 + (y - cy) ** 2) >= R
    return out.astype(np.uint8)


# ---- Philox-4x32-10 ---------------------------------------------------------------
_U32 = np.uint64(0xFFFFFFFF)
_PHILOX_MUL = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
_PHILOX_WEYL = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))


def philox4x32_10(ctr, key):
    """Philox-4x32 with 10 rounds.  ctr: four equal-shape arrays (or ints) of
    32-bit counter words; key: two 32-bit key words.  Each round multiplies
    counter words 0 and 2 by the two multipliers into 64-bit products and
    forms (hi(p1) ^ c1 ^ k0, lo(p1), hi(p0) ^ c3 ^ k1, lo(p0)); the key is
    bumped by the two Weyl constants between rounds.  Returns the four output
    words as uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _U32 for c in ctr)
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + _PHILOX_WEYL[0]) & _U32
            k1 = (k1 + _PHILOX_WEYL[1]) & _U32
        p0 = _PHILOX_MUL[0] * c0
        p1 = _PHILOX_MUL[1] * c2
        c0, c1, c2, c3 = (p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & _U32, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & _U32
    return c0, c1, c2, c3


def philox_noise(seed: int, instance: int, N: int, amp: float) -> np.ndarray:
    """The continuation noise of ttsh_reseed for destination `instance`,
    [2][N][N] float64: key = (seed mod 2^32, seed >> 32), counter = (i N + j,
    instance, 0, 0) for node (i, j); output word c gives component c as
    amp (2 u - 1) with u = (word >> 8) 2^-24, evaluated in FP64 (exact up to
    the final multiplication by amp)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    idx = np.arange(N * N, dtype=np.uint64).reshape(N, N)
    w = philox4x32_10((idx, np.uint64(instance), np.uint64(0), np.uint64(0)), (seed & 0xFFFFFFFF, seed >> 32))
    out = np.empty((2, N, N))
    for c in range(2):
        u = (w[c] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
        out[c] = amp * (2.0 * u - 1.0)
    return out


@dataclasses.dataclass(frozen=True)
class Coefficients:
    """Coefficients of the general form L(k) = -alpha - Gamma0 k^2 - Gamma2 k^4
    with cubic (beta), advection (lambda0, lambda1) and mask (gamma_v,
    gamma_w) terms, the time step and the stepper.  Defaults: the workloads'
    set (alpha = -1, beta = 1, Gamma0 = -1, Gamma2 = 1, lambda0 = 3,
    lambda1 = 0, one penalisation 100 on the velocity, none on the
    vorticity, dt = 0.01, integrating-factor Euler)."""
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


def workload_coefficients(dt: float = 0.01) -> Coefficients:
    return Coefficients(dt=dt)


def paper_coefficients(dt: float = 0.01) -> Coefficients:
    """The paper's preset (a, b, lambda, gamma_v, gamma_w) = (0.5, 1.6, 9, 40, 4)
    in the general form: alpha = 1 - a, Gamma0 = -2, Gamma2 = 1 (model
    subsection; Table I)."""
    return Coefficients(alpha=0.5, beta=1.6, gamma0=-2.0, gamma2=1.0, lambda0=9.0, lambda1=0.0,
                        gamma_v=40.0, gamma_w=4.0, dt=dt)


@dataclasses.dataclass
class Instance:
    N: int
    L: float
    centers: List[Tuple[float, float]]
    radii: List[float]
    xi: float
    seed: int


@dataclasses.dataclass
class Workload:
    name: str
    precision: int
    dt: float
    steps: int
    instances: List[Instance]
    note: str = ""

    @property
    def points(self) -> int:
        return sum(i.N * i.N for i in self.instances)


def circle_fp64_64() -> Workload:
    """64 x 64 box of side 64, one circle R = 8 (tanh width 0.5), FP64, 2000 steps."""
    return Workload("circle64_fp64", 64, 0.01, 2000,
                    [Instance(64, 64.0, [(0.0, 0.0)], [8.0], 0.5, 0)])


def circle_fp32_512() -> Workload:
    """512 x 512 box of side 256, one circle R = 60, FP32, 1e5 steps (the
    comparison with the FP64 oracle is taken at step 1000)."""
    return Workload("circle512_fp32", 32, 0.01, 100_000,
                    [Instance(512, 256.0, [(0.0, 0.0)], [60.0], 0.5, 1)])


def sweep_size(R: float) -> Tuple[int, float]:
    """Box side L = 3.2 R and the smallest N in {128, 256, 512} with L/N <= 0.5."""
    L = 3.2 * R
    for N in (128, 256, 512):
        if L / N <= 0.5 + 1e-12:
            return N, L
    return 512, L


def radius_sweep(n_radii: int = 32) -> Workload:
    """Batched hysteresis sweep: n_radii radii linearly spaced 8..80, each run
    on an upward and a downward ramp (2 n_radii instances), L = 3.2 R, N chosen
    per radius; stage 0 seeds 100 + instance index.  Instance 2j is radius j on
    the upward ramp, 2j+1 the same radius on the downward ramp."""
    inst = []
    for j in range(n_radii):
        R = 8.0 + 72.0 * j / (n_radii - 1)
        N, L = sweep_size(R)
        for ramp in range(2):
            idx = 2 * j + ramp
            inst.append(Instance(N, L, [(0.0, 0.0)], [R], 0.5, 100 + idx))
    return Workload("radius_sweep_fp32", 32, 0.01, 20_000, inst,
                    note="64 instances: 12 x 128^2, 16 x 256^2, 36 x 512^2")


def sweep_chain(n_radii: int = 32):
    """Chain predecessor of each sweep instance for the continuation between
    stages: upward ramp takes radius j-1's final state, downward ramp radius
    j+1's; chain heads continue from their own state.  Returns a list src[i]."""
    src = []
    for j in range(n_radii):
        src.append(2 * (j - 1) if j > 0 else 0)                   # up
        src.append(2 * (j + 1) + 1 if j < n_radii - 1 else 2 * j + 1)  # down
    return src


def dumbbells(n: int = 16, N: int = 1024) -> Workload:
    """Dumbbell geometries: two circles R = 40 with centre distance d linearly
    spaced 40..80, centres (+-d/2, 0), N x N grid of side 256, seeds 300 + i."""
    inst = []
    for i in range(n):
        d = 40.0 + 40.0 * i / (n - 1) if n > 1 else 40.0
        inst.append(Instance(N, 256.0, [(-d / 2, 0.0), (d / 2, 0.0)], [40.0, 40.0], 0.5, 300 + i))
    return Workload("dumbbell1024_fp32", 32, 0.01, 50_000, inst)


def stage_seed(stage: int) -> int:
    """Seed of the continuation noise drawn after stage `stage` (the noise of
    each destination instance is told apart by its index in the counter)."""
    return 1_000_003 * (stage + 1)
