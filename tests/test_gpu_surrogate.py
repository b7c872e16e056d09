"""The surrogate end to end on the GPU: data from solver trajectories, a
short training run of the network by the library's own forward/backward/Adam
kernels, what the trained network gains over the method without it, and the
rollout's acceptance checks and solver fallback.

Instances: the six smallest radii of the radius sweep (R = 8 .. 19.6, both
ramps, native grid 128^2, box L = 3.2 R), recorded every 20 solver steps
after 400 steps (the decay of the initial noise is over by then; the data
hold the growth of the unstable band and the formation of the confined
flow).  Radius j = 3 (both ramps) is held out."""
import numpy as np
import pytest

from oracle import ttsh as O
from paper_2304_03306_amd import workloads as W

pytestmark = pytest.mark.gpu

N_RADII = 6
N_SNAP = 100
EVERY = 20
TRANSIENT = 400
HELD_OUT = [6, 7]


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def data(gpu):
    from paper_2304_03306_amd import surrogate as S
    say("surrogate data", N_RADII, "radii x 2 ramps,", N_SNAP, "snapshots every", EVERY)
    inst = W.radius_sweep().instances[:2 * N_RADII]
    assert all(i.N == 128 for i in inst)
    p = O.workload_params()
    masks = S.coarse_masks(inst, 128, p)
    solver = S.new_solver(inst, p)
    D = S.collect(solver, masks, N_SNAP, EVERY, 128, transient=TRANSIENT)
    return dict(inst=inst, p=p, masks=masks, solver=solver, D=D)


def test_collected_snapshots_are_the_solver_trajectory(data, gpu):
    """Snapshot t of instance i is the solver's field after TRANSIENT +
    t*EVERY steps (a fresh run of the same instance reproduces it bit for
    bit), and channel 2 is the coarse mask."""
    import torch
    from paper_2304_03306_amd import surrogate as S
    say("surrogate snapshots vs fresh run")
    D = data["D"]
    assert torch.equal(D[5, :, :, :, 2].cpu(), torch.from_numpy(data["masks"]))
    s = S.new_solver(data["inst"][2:3], data["p"])
    s.step(TRANSIENT + 5 * EVERY)
    buf = torch.zeros((128, 128, 3), dtype=torch.float32, device="cuda")
    s.field_coarse(0, 128, buf, 3)
    assert torch.equal(buf[..., :2], D[5, 2, :, :, :2])


@pytest.fixture(scope="module")
def trained(data, gpu):
    from paper_2304_03306_amd import surrogate as S
    say("surrogate training (time-limited)")
    # the plain training set (no symmetry augmentation), the configuration
    # whose gain the test below bounds
    cfg = S.SurrogateConfig(batch=64, lr=3e-3, augment=False)
    tr = S.Trainer(cfg, seed=0)
    train_ids = [i for i in range(2 * N_RADII) if i not in HELD_OUT]
    hist = tr.train(data["D"], train_ids, epochs=300, seed=1, log=lambda m: print(m, flush=True),
                    time_limit=90.0)
    return tr, hist


def test_trained_network_beats_persistence(data, trained):
    """What the trained network gains: on held-out radii its one-step
    prediction (projected) is at least 30 % closer to the solver than the
    field left unchanged (persistence; measured: about 45 % closer), and
    training at least halved the loss.  (Normalising the loss by the change
    over the step instead, fno_loss_ex, gave 0.062 against 0.070 here: the
    plain relative error of the field is the better training loss.)"""
    from paper_2304_03306_amd import surrogate as S
    tr, hist = trained
    assert hist[-1][1] < 0.5 * hist[0][1], hist
    ev = tr.eval_one_step(data["D"], HELD_OUT, project=data["solver"])
    print("held-out one-step errors", ev, flush=True)
    assert np.isfinite(ev["network_projected"])
    assert ev["network_projected"] <= ev["network"] * (1 + 1e-3)
    assert ev["network_projected"] < 0.7 * ev["persistence"], ev


def test_rollout_is_checked_and_falls_back(data, trained):
    """A rollout over all instances: per-step errors against the recorded
    solver trajectory are finite; with corrupted weights every instance fails
    acceptance at the first step and continues on the solver, so its error
    stays that of the coarse restart (small)."""
    import torch
    from paper_2304_03306_amd import surrogate as S
    say("surrogate rollout + fallback")
    tr, _ = trained
    D = data["D"]
    t0, steps = 40, 20
    reference = lambda s: D[t0 + s] if t0 + s < D.shape[0] else None
    ro = S.Rollout(tr.net, tr.cfg, data["inst"], data["p"], data["solver"], check_every=10, tol=0.2)
    res = ro.run(D[t0], steps, reference=reference, log=lambda m: print(m, flush=True))
    print("rollout mean err per step", np.nanmean(res.err, axis=1), "fallbacks", res.fallback_step, flush=True)
    assert np.isfinite(res.err).all()
    # corrupted weights -> non-finite output -> all instances on the solver
    good = tr.net.params()
    bad = good.copy()
    bad[: bad.size // 2] = np.nan
    tr.net.set_params(bad)
    try:
        res2 = ro.run(D[t0], 5, reference=reference)
    finally:
        tr.net.set_params(good)
    assert (res2.fallback_step == 0).all(), res2.fallback_step
    assert all(r == "non-finite" for r in res2.reason)
    assert np.isfinite(res2.err).all() and res2.err.max() < 0.05, res2.err


def test_scale_channel_pipeline(data):
    """With the grid-spacing channel the snapshots carry L/Nc as a constant
    fourth channel beside the same (v_x, v_y, K); a 4-input network trains a
    few batches and rolls out with finite errors."""
    import torch
    from paper_2304_03306_amd import surrogate as S
    say("surrogate scale channel")
    inst = data["inst"][:4]
    masks = data["masks"][:4]
    s = S.new_solver(inst, data["p"])
    spacing = [i.L / 128 for i in inst]
    D4 = S.collect(s, masks, 6, EVERY, 128, transient=TRANSIENT, spacing=spacing)
    assert D4.shape[-1] == 4
    for i in range(4):
        assert torch.all(D4[:, i, :, :, 3] == np.float32(spacing[i]))
    ref = data["D"][:6, :4]
    assert float((D4[..., :3] - ref).norm() / ref.norm()) < 1e-5  # same trajectories (tuning may reorder sums)
    cfg = S.SurrogateConfig(batch=8, cin=4)
    tr = S.Trainer(cfg, seed=0)
    hist = tr.train(D4, [0, 1, 2, 3], epochs=2, seed=1)
    assert np.isfinite(hist[-1][1])
    ro = S.Rollout(tr.net, cfg, inst, data["p"], s, check_every=0, envelope=float("inf"))
    res = ro.run(D4[0], 3, reference=lambda k: D4[k] if k < D4.shape[0] else None)
    assert np.isfinite(res.err).all()


def test_pushforward_batch_trains_on_the_networks_own_prediction(data, gpu):
    """A pushforward batch's input is the network's one-step prediction of
    snapshot t from snapshot t - 1 (velocity channels; the mask channel is the
    snapshot's), made with the weights before the step, and its target is
    snapshot t + 1; the step is then an ordinary Adam step (the loss is finite
    and the weights change).  Inputs at the first snapshot are moved to the
    second by the schedule, so every index has a predecessor."""
    import torch
    from paper_2304_03306_amd import surrogate as S
    say("surrogate pushforward batch")
    D = data["D"]
    I = D.shape[1]
    cfg = S.SurrogateConfig(batch=8, lr=1e-3, augment=False, pushforward=1.0, pushforward_start=0.0)
    tr = S.Trainer(cfg, seed=3)
    idx = np.array([5 * I + 0, 7 * I + 3, 1 * I + 4, 40 * I + 11], dtype=np.int64)
    B = len(idx)
    x = torch.empty((B, 128, 128, 3), dtype=torch.float32, device="cuda")
    tr.net.gather(x, 3, D, D.shape[-1], 3, 128 * 128, idx - I)
    want = x.clone()
    tr.net.forward_ex(want, want, 3, True, B)
    p0 = tr.net.params().copy()
    loss = tr.batch_step(D, idx, 1e-3, pushforward=True)
    assert np.isfinite(loss)
    assert torch.equal(tr.xb[:B], want)
    assert torch.equal(tr.xb[:B, ..., 2], D.view(-1, 128, 128, 3)[torch.from_numpy(idx).cuda()][..., 2])
    assert torch.equal(tr.tb[:B], D.view(-1, 128, 128, 3)[torch.from_numpy(idx + I).cuda()][..., :2])
    assert not np.array_equal(tr.net.params(), p0)
    hist = tr.train(D[:4], [0, 1], epochs=2, seed=5)  # every batch pushforward, first-snapshot inputs moved
    assert all(np.isfinite(h[1]) for h in hist)
