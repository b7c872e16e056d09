"""Coarse-field surrogate of the solver: training data from solver
trajectories, training of the Fourier neural operator (libttsh's fno_* entry
points), and rollout with acceptance checks, solver fallback and the solver
as the reference for its error.

Every arithmetic step runs in the HIP library: the solver (ttsh_*), the
coarsening and its inverse (ttsh_get_field_coarse / ttsh_set_field_coarse),
the projection of the network's output (ttsh_project_coarse), the network
(fno_*) and the per-sample errors (fno_sample_errors).  This module only
orders the calls, moves buffers and keeps host-side bookkeeping (sample
indices, learning-rate schedule, acceptance decisions).

Data layout on the device: snapshots D[t][i] of instance i at surrogate step
t, each a channels-last float32 Nc x Nc x cin field (v_x, v_y, K[, dx]), where
K is the instance's mask sampled on the coarse grid and the optional fourth
channel holds the coarse grid spacing L/Nc of the instance's box as a
constant (the radius sets the box, so this tells the network the physical
scale the coarse fields are on).  One surrogate step advances
`every` solver steps.  The network predicts the change of (v_x, v_y) over one
surrogate step (residual output), and the rollout projects each prediction
onto the coarse solver's state space (1/2-rule cutoff, divergence-free) as a
hard constraint.
"""
from __future__ import annotations

import dataclasses
import math
import os
import time
from typing import List, Optional, Sequence

import numpy as np

from . import fno as F
from . import ttsh as T
from .workloads import Instance, uniform_field


@dataclasses.dataclass
class SurrogateConfig:
    Nc: int = 128          # coarse grid
    every: int = 20        # solver steps per surrogate step
    width: int = 32
    modes: int = 16
    layers: int = 4
    hidden: int = 128
    batch: int = 256
    lr: float = 1e-3
    cin: int = 3           # v_x, v_y, K (4: and the grid spacing, see scale_channel)
    cout: int = 2
    increment_loss: bool = False  # normalise the loss by the change over the step (fno_loss_ex)
    input_noise: float = 0.0      # uniform perturbation of the input velocity in training
    augment: bool = True          # a random symmetry of the square per training sample (fno_gather_d4)
    # pushforward training: this fraction of the batches, from pushforward_start of the
    # schedule on, takes as input the network's own prediction of the snapshot from the
    # one before it (no gradient through that prediction), so that the network learns to
    # correct the errors its rollouts feed back to it
    pushforward: float = 0.0
    pushforward_start: float = 0.25


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the surrogate runs on the GPU only")
    return torch


def coarse_masks(instances: Sequence[Instance], Nc: int, params) -> np.ndarray:
    """Masks of the instances sampled on the coarse grid (same box, same
    circles and width), computed by the library; float32 [I][Nc][Nc]."""
    s = T.Solver([Nc] * len(instances), [inst.L for inst in instances], params, T.TTSH_FP32)
    try:
        out = np.empty((len(instances), Nc, Nc), dtype=np.float32)
        for i, inst in enumerate(instances):
            s.mask_tanh(i, inst.centers, inst.radii, inst.xi)
            out[i] = s.mask(i)
        return out
    finally:
        s.close()


def new_solver(instances: Sequence[Instance], params, precision=T.TTSH_FP32, seed_fields=True,
               graph_steps: int = 20, tune: bool = True) -> T.Solver:
    """A solver context over the instances, masks set, started from each
    instance's seeded initial field; steps are replayed from graphs of
    graph_steps steps (one surrogate step's worth)."""
    s = T.Solver([i.N for i in instances], [i.L for i in instances], params, precision)
    s.option(T.TTSH_OPT_GRAPH_STEPS, graph_steps)
    for q, inst in enumerate(instances):
        s.mask_tanh(q, inst.centers, inst.radii, inst.xi)
        if seed_fields:
            s.set_field(q, uniform_field(inst.seed, inst.N, 0.01, precision))
    if tune:
        s.tune(graph_steps)  # workgroup sizes per pass; the state is restored
    return s


def snapshot(solver: T.Solver, n_inst: int, Nc: int, out) -> None:
    """Write every instance's coarse velocity into channels 0..1 of out
    [I][Nc][Nc][cin] (float32 device tensor)."""
    cin = out.shape[-1]
    for i in range(n_inst):
        solver.field_coarse(i, Nc, out[i], cin)


def collect(solver: T.Solver, masks: np.ndarray, n_snap: int, every: int, Nc: int, transient: int = 0,
            log=None, spacing: Optional[Sequence[float]] = None):
    """Run the solver and record n_snap snapshots, `every` steps apart, after
    `transient` steps.  Returns a device tensor D [n_snap][I][Nc][Nc][cin]
    with cin = 3, or 4 when the coarse grid spacings of the instances are
    given (a constant fourth channel)."""
    torch = _torch()
    I = masks.shape[0]
    cin = 3 if spacing is None else 4
    D = torch.empty((n_snap, I, Nc, Nc, cin), dtype=torch.float32, device="cuda")
    Kd = torch.from_numpy(masks).cuda()
    if spacing is not None:
        hd = torch.tensor(np.asarray(spacing, dtype=np.float32), device="cuda")[:, None, None].expand(I, Nc, Nc)
    if transient:
        solver.step(transient)
    t0 = time.time()
    for t in range(n_snap):
        D[t, :, :, :, 2] = Kd
        if spacing is not None:
            D[t, :, :, :, 3] = hd
        snapshot(solver, I, Nc, D[t])
        if t + 1 < n_snap:
            solver.step(every)
        if log and (t + 1) % 100 == 0:
            solver.sync()
            log(f"collect {t + 1}/{n_snap} snapshots, {time.time() - t0:.1f} s")
    solver.sync()
    return D


def split_by_radius(n_radii: int, hold_every: int = 4):
    """Train/test split of the radius sweep by radius: every hold_every-th
    radius (both ramps) is held out.  Returns (train_ids, test_ids)."""
    test = [2 * j + r for j in range(n_radii) if j % hold_every == hold_every - 1 for r in (0, 1)]
    train = [i for i in range(2 * n_radii) if i not in test]
    return train, test


class Trainer:
    """Adam training of one network on snapshot pairs (D[t][i], D[t+1][i])."""

    def __init__(self, cfg: SurrogateConfig, seed: int = 0):
        torch = _torch()
        self.cfg = cfg
        self.net = F.FNO(width=cfg.width, modes=cfg.modes, layers=cfg.layers, cin=cfg.cin, cout=cfg.cout,
                         hidden=cfg.hidden, H=cfg.Nc, W=cfg.Nc, max_batch=cfg.batch, seed=seed)
        n = cfg.Nc
        self.xb = torch.empty((cfg.batch, n, n, cfg.cin), dtype=torch.float32, device="cuda")
        self.tb = torch.empty((cfg.batch, n, n, cfg.cout), dtype=torch.float32, device="cuda")
        self.yb = torch.empty_like(self.tb)
        self.step_count = 0
        self.rng = np.random.default_rng(seed + 7919)  # the augmentation's symmetry elements

    def pairs(self, D, ids: Sequence[int]) -> np.ndarray:
        """Flat sample indices (into D viewed as [n_snap * I]) of every input
        whose successor exists."""
        n_snap, I = D.shape[0], D.shape[1]
        return np.array([t * I + i for t in range(n_snap - 1) for i in ids], dtype=np.int64)

    def batch_step(self, D, idx: np.ndarray, lr: float, pushforward: bool = False) -> float:
        """One Adam step on the pairs idx -> idx + I.  With pushforward every
        idx must have a predecessor (idx >= I): the input is then the
        network's one-step prediction from snapshot idx - I, formed in place
        by an inference forward (the mask and spacing channels are those of
        the snapshot, which do not change along a trajectory)."""
        c = self.cfg
        I = D.shape[1]
        npix = c.Nc * c.Nc
        B = len(idx)
        dch = D.shape[-1]
        src = idx - I if pushforward else idx
        if c.augment:
            # the same rotation or reflection for a sample's input and target
            sym = self.rng.integers(0, 8, B)
            self.net.gather_d4(self.xb, c.cin, D, dch, c.cin, c.Nc, src, sym)
            self.net.gather_d4(self.tb, c.cout, D, dch, c.cout, c.Nc, idx + I, sym)
        else:
            self.net.gather(self.xb, c.cin, D, dch, c.cin, npix, src)
            self.net.gather(self.tb, c.cout, D, dch, c.cout, npix, idx + I)
        if pushforward:
            self.net.forward_ex(self.xb, self.xb, c.cin, True, B)
        if c.input_noise > 0:
            self.net.perturb(self.xb, c.cin, c.cout, B * npix, c.input_noise, self.step_count + 1)
        self.net.forward_ex(self.xb, self.yb, c.cout, True, B, train=True)
        if c.increment_loss:
            loss = self.net.loss_ex(self.yb, self.tb, self.xb, c.cin, B)
        else:
            loss = self.net.loss(self.yb[:B], self.tb[:B])
        self.net.backward(B)
        self.net.adam_step(lr)
        self.step_count += 1
        return loss

    def train(self, D, ids: Sequence[int], epochs: int, seed: int = 0, log=None, time_limit: float = None):
        """Cosine-decayed Adam over `epochs` passes of the shuffled pairs.
        Returns the list of (epoch, mean loss, seconds)."""
        c = self.cfg
        pairs = self.pairs(D, ids)
        I = D.shape[1]
        if c.pushforward > 0 and D.shape[0] < 3:
            raise ValueError("pushforward training needs at least three snapshots")
        rng = np.random.default_rng(seed)
        nb = max(1, len(pairs) // c.batch)
        total = epochs * nb
        hist = []
        t0 = time.time()
        k = 0
        for ep in range(epochs):
            perm = rng.permutation(pairs)
            acc = 0.0
            for b in range(nb):
                lr = 0.5 * c.lr * (1.0 + math.cos(math.pi * k / total))
                idx = perm[b * c.batch:(b + 1) * c.batch]
                pf = c.pushforward > 0 and k >= c.pushforward_start * total and rng.random() < c.pushforward
                if pf:  # inputs at the first snapshot have no predecessor: take the next pair instead
                    idx = np.where(idx < I, idx + I, idx)
                acc += self.batch_step(D, idx, lr, pushforward=pf)
                k += 1
            hist.append((ep, acc / nb, time.time() - t0))
            if log and (ep % 10 == 0 or ep == epochs - 1):
                log(f"epoch {ep} loss {acc / nb:.4e} ({time.time() - t0:.1f} s)")
            if time_limit is not None and time.time() - t0 > time_limit:
                break
        return hist

    def eval_one_step(self, D, ids: Sequence[int], project: Optional[T.Solver] = None):
        """Mean relative L2 error of one surrogate step over the pairs of
        `ids` (full-field error of the predicted velocity), with and without
        projecting the prediction, and of persistence (v(t + 1) = v(t))."""
        torch = _torch()
        c = self.cfg
        pairs = self.pairs(D, ids)
        I = D.shape[1]
        npix = c.Nc * c.Nc
        errs, errs_p, pers = [], [], []
        xb = torch.empty((c.batch, c.Nc, c.Nc, c.cin), dtype=torch.float32, device="cuda")
        for b0 in range(0, len(pairs), c.batch):
            idx = pairs[b0:b0 + c.batch]
            B = len(idx)
            self.net.gather(xb, c.cin, D, D.shape[-1], c.cin, npix, idx)
            self.net.gather(self.tb, c.cout, D, D.shape[-1], c.cout, npix, idx + I)
            pers.append(F.fno_sample_errors(xb, c.cin, self.tb, c.cout, c.cout, npix, B))
            self.net.forward_ex(xb, self.yb, c.cout, True, B)
            errs.append(F.fno_sample_errors(self.yb, c.cout, self.tb, c.cout, c.cout, npix, B))
            if project is not None:
                self.net.forward_ex(xb, xb, c.cin, True, B)
                project.project_coarse(c.Nc, xb, c.cin, B)
                errs_p.append(F.fno_sample_errors(xb, c.cin, self.tb, c.cout, c.cout, npix, B))
        out = dict(network=float(np.mean(np.concatenate(errs))), persistence=float(np.mean(np.concatenate(pers))))
        if errs_p:
            out["network_projected"] = float(np.mean(np.concatenate(errs_p)))
        return out


@dataclasses.dataclass
class RolloutResult:
    err: np.ndarray            # [steps][I] rel-L2 vs the reference (NaN where none)
    fallback_step: np.ndarray  # [I] surrogate step at which the instance went to the solver (-1: never)
    reason: List[str]
    seconds: float             # wall time of the rollout (surrogate + checks + fallback)
    seconds_surrogate: float   # of which network + projection + acceptance


class Rollout:
    """Advance coarse fields with the network; hand an instance back to the
    native-grid solver when its prediction fails an acceptance test.

    Acceptance, per instance and surrogate step: every value finite, and the
    energy sum |v|^2 and enstrophy sum |w|^2 of the projected prediction
    within a factor `envelope` of the previous step's.  Every `check_every`
    steps the solver checks the network locally: the current coarse fields
    are put on the native grids, advanced `every` solver steps and coarsened;
    if the network's prediction from the same fields is further than `tol`
    (relative L2) from that, the instance fails too.  A failed instance
    continues with the solver, on its native grid, from its last accepted
    coarse field (the field the failed step started from).  The context
    `checker` (all instances) serves the checks and the projection; the
    solver runs of failed instances get contexts of their own."""

    def __init__(self, net: F.FNO, cfg: SurrogateConfig, instances: Sequence[Instance], params,
                 checker: T.Solver, envelope: float = 1.5, check_every: int = 25, tol: float = 0.1):
        self.net, self.cfg, self.inst, self.params = net, cfg, list(instances), params
        self.checker = checker
        self.envelope, self.check_every, self.tol = envelope, check_every, tol

    def run(self, x0, steps: int, reference=None, log=None) -> RolloutResult:
        """x0: device [I][Nc][Nc][cin] (v_x, v_y, K[, dx]) at surrogate step 0.
        reference(s) -> device [I][Nc][Nc][>=2] solver fields at step s, or None."""
        torch = _torch()
        c = self.cfg
        I = x0.shape[0]
        ch = x0.shape[-1]  # pixel stride of the coarse fields
        npix = c.Nc * c.Nc
        x = x0.clone()
        x_prev = torch.empty_like(x)
        ref = torch.empty_like(x)
        err = np.full((steps, I), np.nan)
        fb_step = np.full(I, -1)
        reason = [""] * I
        active = np.ones(I, dtype=bool)
        solvers = []  # (context, instance ids) of instances on the solver
        prev = None
        t_sur = 0.0
        torch.cuda.synchronize()
        t0 = time.time()
        for s in range(steps):
            check = self.check_every > 0 and s % self.check_every == 0 and active.any()
            x_prev.copy_(x)
            if check:
                ids = np.flatnonzero(active)
                for i in ids:
                    self.checker.set_field_coarse(int(i), c.Nc, x[i], ch)
                self.checker.step(c.every)
                for i in ids:
                    self.checker.field_coarse(int(i), c.Nc, ref[i], ch)
            ts = time.time()
            self.net.forward_ex(x, x, ch, True, I)
            nrm = self.checker.project_coarse(c.Nc, x, ch, I, norms=True)
            t_sur += time.time() - ts
            bad = ~np.isfinite(nrm).all(axis=1)
            fail = active & bad
            if prev is not None:
                with np.errstate(divide="ignore", invalid="ignore"):
                    ratio = nrm / prev
                out_env = ~((ratio <= self.envelope) & (ratio >= 1.0 / self.envelope)).all(axis=1)
                fail |= active & ~bad & out_env
            for i in np.flatnonzero(fail):
                reason[i] = "non-finite" if bad[i] else "energy/enstrophy envelope"
            if check:
                e_loc = F.fno_sample_errors(x, ch, ref, ch, 2, npix, I)
                loc = active & ~fail & ~(e_loc <= self.tol)
                for i in np.flatnonzero(loc):
                    reason[i] = f"local check {e_loc[i]:.3g} > {self.tol}"
                fail |= loc
            if fail.any():
                ids = [int(i) for i in np.flatnonzero(fail)]
                fb_step[ids] = s
                active[ids] = False
                sol = new_solver([self.inst[i] for i in ids], self.params, seed_fields=False)
                for q, i in enumerate(ids):
                    sol.set_field_coarse(q, c.Nc, x_prev[i], ch)
                solvers.append((sol, ids))
                if log:
                    log(f"step {s}: instances {ids} -> solver ({reason[ids[0]]})")
            for sol, ids in solvers:
                sol.step(c.every)
                for q, i in enumerate(ids):
                    sol.field_coarse(q, c.Nc, x[i], ch)
            prev = nrm if prev is None else np.where(active[:, None], nrm, prev)
            if reference is not None:
                tgt = reference(s + 1)
                if tgt is not None:
                    err[s] = F.fno_sample_errors(x, ch, tgt, tgt.shape[-1], 2, npix, I)
            if log and (s + 1) % 50 == 0:
                log(f"rollout step {s + 1}/{steps}: mean err {np.nanmean(err[s]):.3e}, "
                    f"{int(active.sum())} on the network")
        torch.cuda.synchronize()
        secs = time.time() - t0
        for sol, _ in solvers:
            sol.close()
        return RolloutResult(err, fb_step, reason, secs, t_sur)


def solver_step_seconds(solver: T.Solver, every: int, reps: int = 20) -> float:
    """Wall seconds for `every` solver steps of the whole context (graph
    replays, device-synchronised)."""
    torch = _torch()
    solver.step(every)
    solver.sync()
    t0 = time.time()
    for _ in range(reps):
        solver.step(every)
    solver.sync()
    torch.cuda.synchronize()
    return (time.time() - t0) / reps


def surrogate_step_seconds(net: F.FNO, checker: T.Solver, x, Nc: int, reps: int = 20) -> float:
    """Wall seconds of one surrogate step for the batch x (inference forward
    with residual output in place, projection with the acceptance norms)."""
    torch = _torch()
    y = x.clone()
    B, ch = x.shape[0], x.shape[-1]
    net.forward_ex(y, y, ch, True, B)
    checker.project_coarse(Nc, y, ch, B, norms=True)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(reps):
        net.forward_ex(y, y, ch, True, B)
        checker.project_coarse(Nc, y, ch, B, norms=True)
    torch.cuda.synchronize()
    return (time.time() - t0) / reps


def first_exceeding(curve: np.ndarray, thr: float) -> int:
    """Index of the first entry above thr (len(curve) if none)."""
    above = np.flatnonzero(~(curve <= thr))
    return int(above[0]) if above.size else len(curve)


def main(argv=None):
    """Radius-sweep surrogate: collect, train, roll out, compare with the solver; one JSON report."""
    import argparse
    import json
    from . import workloads as Wl
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--transient", type=int, default=2000, help="solver steps before the first snapshot")
    ap.add_argument("--snapshots", type=int, default=1001)
    ap.add_argument("--train-until", type=int, default=500, help="pairs with t < this are training data")
    ap.add_argument("--rollout", type=int, default=500, help="surrogate steps of the rollout")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--train-seconds", type=float, default=300.0)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--modes", type=int, default=16)
    ap.add_argument("--input-noise", type=float, default=0.0)
    ap.add_argument("--scale-channel", action="store_true",
                    help="a fourth input channel with the coarse grid spacing L/Nc of each instance")
    ap.add_argument("--no-augment", action="store_true",
                    help="train without the random rotation or reflection of the square per sample (by default "
                         "each training sample takes one: the circles sit on the grid centre, and the equation "
                         "has no preferred direction or handedness)")
    ap.add_argument("--pushforward", type=float, default=0.0,
                    help="fraction of the training batches (after the first quarter of the schedule) whose input "
                         "is the network's own one-step prediction from the previous snapshot")
    ap.add_argument("--threshold", type=float, default=0.1)
    ap.add_argument("--check-every", type=int, default=25)
    ap.add_argument("--report", default="surrogate_report.json")
    ap.add_argument("--speed-only", action="store_true",
                    help="only time one surrogate step against the solver's 20 steps (untrained weights)")
    a = ap.parse_args(argv)
    torch = _torch()
    log = lambda m: print(f"[surrogate] {m}", flush=True)
    wl = Wl.radius_sweep()
    inst = wl.instances
    params = Wl.workload_coefficients()
    cfg = SurrogateConfig(batch=a.batch, lr=a.lr, modes=a.modes, input_noise=a.input_noise,
                          cin=4 if a.scale_channel else 3, augment=not a.no_augment, pushforward=a.pushforward)
    I, Nc = len(inst), cfg.Nc
    spacing = [i.L / Nc for i in inst] if a.scale_channel else None
    masks = coarse_masks(inst, Nc, params)
    solver = new_solver(inst, params)
    if a.speed_only:
        D = collect(solver, masks, 1, cfg.every, Nc, transient=a.transient, spacing=spacing)
        net = F.FNO(width=cfg.width, modes=cfg.modes, layers=cfg.layers, cin=cfg.cin, cout=cfg.cout,
                    hidden=cfg.hidden, H=Nc, W=Nc, max_batch=I, seed=0)
        t_sur = surrogate_step_seconds(net, solver, D[0], Nc)
        t_sol = solver_step_seconds(solver, cfg.every)
        log(f"surrogate step {t_sur * 1e3:.3f} ms, {cfg.every} solver steps {t_sol * 1e3:.3f} ms: "
            f"{t_sol / t_sur:.2f}x")
        return {"seconds_per_surrogate_step": t_sur, "seconds_per_solver_steps": t_sol}
    log(f"{I} instances, transient {a.transient} steps, {a.snapshots} snapshots every {cfg.every}")
    D = collect(solver, masks, a.snapshots, cfg.every, Nc, transient=a.transient, log=log, spacing=spacing)
    train_ids, test_ids = split_by_radius(I // 2)
    # training pairs: snapshots 0 .. train_until (the rollout starts after them)
    tr = Trainer(cfg, seed=0)
    Dtrain = D[:a.train_until + 1]
    hist = tr.train(Dtrain, train_ids, a.epochs, seed=1, log=log, time_limit=a.train_seconds)
    log(f"trained {len(hist)} epochs in {hist[-1][2]:.0f} s, loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
    t0 = a.train_until
    Deval = D[t0:]
    one = {"test": tr.eval_one_step(Deval, test_ids, project=solver),
           "train_radii_later_times": tr.eval_one_step(Deval, train_ids, project=solver)}
    log(f"one-step errors after the training window: {one}")
    steps = min(a.rollout, D.shape[0] - 1 - t0)
    reference = lambda s: D[t0 + s] if t0 + s < D.shape[0] else None
    # pure network (no checks), then with acceptance checks and fallback
    ro_free = Rollout(tr.net, cfg, inst, params, solver, envelope=float("inf"), check_every=0)
    free = ro_free.run(D[t0], steps, reference=reference, log=log)
    ro = Rollout(tr.net, cfg, inst, params, solver, check_every=a.check_every, tol=a.threshold)
    guarded = ro.run(D[t0], steps, reference=reference, log=log)
    # persistence for reference
    npix = Nc * Nc
    dch = D.shape[-1]
    pers = np.stack([F.fno_sample_errors(D[t0], dch, D[t0 + s + 1], dch, 2, npix, I) for s in range(steps)])
    t_sur = surrogate_step_seconds(tr.net, solver, D[t0], Nc)
    t_sol = solver_step_seconds(solver, cfg.every)
    test = np.array(test_ids)
    curve = np.nanmean(free.err[:, test], axis=1)
    s_star = first_exceeding(curve, a.threshold)
    rep = {
        "instances": I, "coarse_grid": Nc, "solver_steps_per_surrogate_step": cfg.every,
        "network": dict(width=cfg.width, modes=cfg.modes, layers=cfg.layers, hidden=cfg.hidden,
                        params=int(tr.net.n), dtype="bf16 storage, fp32 accumulation",
                        input_noise=cfg.input_noise, augment=cfg.augment, pushforward=cfg.pushforward,
                        inputs="v_x, v_y, K" + (", dx" if a.scale_channel else "")),
        "data": dict(transient=a.transient, snapshots=a.snapshots, train_pairs=len(tr.pairs(Dtrain, train_ids)),
                     train_instances=train_ids, test_instances=test_ids),
        "training": dict(epochs=len(hist), seconds=hist[-1][2], loss_first=hist[0][1], loss_last=hist[-1][1],
                         batch=cfg.batch, lr=cfg.lr, schedule="cosine"),
        "one_step": one,
        "rollout_test_mean_err": curve.tolist(),
        "rollout_train_mean_err": np.nanmean(free.err[:, train_ids], axis=1).tolist(),
        "persistence_test_mean_err": pers[:, test].mean(axis=1).tolist(),
        "threshold": a.threshold,
        "steps_within_threshold": s_star,
        "solver_steps_within_threshold": s_star * cfg.every,
        "guarded": dict(fallback_step=guarded.fallback_step.tolist(), reason=guarded.reason,
                        test_mean_err=np.nanmean(guarded.err[:, test], axis=1).tolist(),
                        seconds=guarded.seconds, seconds_network=guarded.seconds_surrogate),
        "seconds_per_surrogate_step": t_sur,
        "seconds_per_solver_20_steps": t_sol,
        "speedup_per_step": t_sol / t_sur,
    }
    os.makedirs(os.path.dirname(os.path.abspath(a.report)), exist_ok=True)
    with open(a.report, "w") as f:
        json.dump(rep, f, indent=1)
    log(f"speedup {t_sol / t_sur:.2f}x per surrogate step ({t_sur * 1e3:.2f} ms vs {t_sol * 1e3:.2f} ms); "
        f"test error stays <= {a.threshold} for {s_star} surrogate steps ({s_star * cfg.every} solver steps)")
    return rep


if __name__ == "__main__":
    main()
