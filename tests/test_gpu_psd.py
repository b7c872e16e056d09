"""Temporal power spectral density of the vorticity on the device
(ttsh_psd_accumulate / ttsh_psd_finish) against the oracle's literal
real-space evaluation of the circle section's definition."""
import numpy as np
import pytest

from oracle import ttsh as O
from paper_2304_03306_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("prec", [64, 32])
def test_psd_matches_oracle(gpu, prec):
    """Three instances (a 64^2 circle, a 128^2 dumbbell, a 512^2 circle)
    sampled 16 times, 25 steps apart: S(f) at frequencies on and off the
    record's grid, negative ones and f = 0 equals the oracle's sum over nodes
    of the same vorticity fields (read back from the states the library
    sampled)."""
    import torch
    say("psd vs oracle", prec)
    Ns, Ls = [64, 128, 512], [32.0, 64.0, 256.0]
    par = O.workload_params()
    s = gpu.Solver(Ns, Ls, par, prec)
    try:
        s.mask_tanh(0, [(0.0, 0.0)], [10.0], 0.5)
        s.mask_tanh(1, [(-10.0, 0.0), (10.0, 0.0)], [12.0, 12.0], 0.5)
        s.mask_tanh(2, [(0.0, 0.0)], [60.0], 0.5)
        for q, N in enumerate(Ns):
            s.set_field(q, W.uniform_field(30 + q, N, 0.1, prec))
        s.step(100)
        T, every = 16, 25
        dts = every * par.dt
        freqs = np.array([0.0, 1 / (T * dts), -1 / (T * dts), 0.37, 1.3, -0.9, 2.0, 0.05])
        accs = [torch.zeros(gpu.psd_buffer_len(N, len(freqs)), dtype=torch.float64, device="cuda") for N in Ns]
        series = [[] for _ in Ns]
        times = []
        for n in range(T):
            t = n * dts
            times.append(t)
            for q, N in enumerate(Ns):
                s.psd_accumulate(q, freqs, t, accs[q])
                vh = O.from_compact(s.state(q), N)
                kx, ky, _, _ = O.grid(N, Ls[q])
                series[q].append(O.field(O.vorticity_hat(vh, kx, ky)[None])[0])
            s.step(every)
        for q, N in enumerate(Ns):
            got = s.psd_finish(N, len(freqs), accs[q])
            want = O.temporal_psd(series[q], times, freqs)
            assert np.max(np.abs(got - want)) < 1e-10 * np.max(want), (q, got, want)
        # a second, differently sized set of frequencies reuses the context's copy
        acc = torch.zeros(gpu.psd_buffer_len(64, 3), dtype=torch.float64, device="cuda")
        s.psd_accumulate(0, [0.1, 0.2, 0.3], 0.5, acc)
        vh = O.from_compact(s.state(0), 64)
        kx, ky, _, _ = O.grid(64, 32.0)
        w = O.field(O.vorticity_hat(vh, kx, ky)[None])[0]
        got = s.psd_finish(64, 3, acc)
        want = O.temporal_psd([w], [0.5], [0.1, 0.2, 0.3])
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(want)
    finally:
        s.close()


def test_psd_rejects_bad_arguments(gpu):
    import torch
    say("psd arguments")
    s = gpu.Solver([64], [32.0], O.workload_params(), 64)
    try:
        acc = torch.zeros(gpu.psd_buffer_len(64, 2), dtype=torch.float64, device="cuda")
        for freqs, t in (([], 0.0), ([0.1, float("nan")], 0.0), ([0.1], float("inf"))):
            with pytest.raises(gpu.TTSHError) as e:
                s.psd_accumulate(0, freqs, t, acc)
            assert e.value.code == gpu.TTSH_EINVAL
        with pytest.raises(gpu.TTSHError) as e:
            s.psd_finish(96, 2, acc)
        assert e.value.code == gpu.TTSH_EUNSUPPORTED
    finally:
        s.close()
