"""The no-allocation continuation entry point against the allocating one:
ttsh_reseed_noalloc (fixed scratch in the library's device memory) must give
the same states as ttsh_reseed, bit for bit, on two calls in a row (the
second with fewer and smaller destinations, so that stale scratch contents
from the first call would show), and refuse requests beyond its scratch."""
import numpy as np
import pytest

from oracle import ttsh as O
from paper_2304_03306_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def make_pair(gpu, Ns, Ls, prec):
    p = O.workload_params()
    out = []
    for _ in range(2):
        s = gpu.Solver(Ns, Ls, p, prec)
        for i, (N, L) in enumerate(zip(Ns, Ls)):
            s.mask_tanh(i, [(0.0, 0.0)], [L / 4], 0.5)
            s.set_field(i, W.uniform_field(90 + i, N, 0.3, prec))
        s.step(3)
        s.sync()
        out.append(s)
    return out


@pytest.mark.parametrize("prec", [64, 32])
def test_reseed_noalloc_equals_reseed(gpu, prec):
    say("reseed noalloc", prec)
    Ns, Ls = [256, 128, 512, 64, 256], [128.0, 64.0, 200.0, 32.0, 128.0]
    a, b = make_pair(gpu, Ns, Ls, prec)
    calls = [([0, 1, 2, 3, 4], [2, 0, 4, 1, 3], 1e-3, 12345),  # every instance, sizes mixed
             ([3, 1], [1, 3], 2e-3, 777)]                       # second call: fewer, smaller
    for dst, src, amp, seed in calls:
        before = [O.from_compact(a.state(i), N) for i, N in enumerate(Ns)]
        gpu.ttsh_reseed(a.ctx, dst, src, amp, seed)
        gpu.ttsh_reseed_noalloc(b.ctx, dst, src, amp, seed)
        b.sync()
        for i in range(len(Ns)):
            assert np.array_equal(a.state(i), b.state(i)), (dst, i)
        # and both are the oracle's continuation
        tol = 1e-12 if prec == 64 else 1e-6
        for d, sr in zip(dst, src):
            want = O.resample(before[sr], Ns[d]) + O.project_field(W.philox_noise(seed, d, Ns[d], amp), Ls[d])
            got = O.from_compact(b.state(d), Ns[d])
            assert np.abs(got - want).max() < tol * np.abs(want).max(), (d, sr)
        # the continued states step on
        a.step(2)
        b.step(2)
        a.sync()
        b.sync()
        for i in range(len(Ns)):
            assert np.array_equal(a.state(i), b.state(i))
    a.close()
    b.close()


def test_reseed_noalloc_refuses_beyond_scratch(gpu):
    """Four 2048^2 destinations need 64.25 MiB of spectra, beyond the 64 MiB
    scratch: refused before any work, the states untouched."""
    say("reseed noalloc limit")
    Ns = [2048] * 4
    s = gpu.Solver(Ns, [64.0] * 4, O.workload_params(), 32)
    s.set_field(0, W.uniform_field(5, 2048, 0.1, 32))
    kept = s.state(0)
    with pytest.raises(gpu.TTSHError) as e:
        gpu.ttsh_reseed_noalloc(s.ctx, [0, 1, 2, 3], [1, 2, 3, 0], 1e-3, 1)
    assert e.value.code == gpu.TTSH_EINVAL and "64 MiB" in str(e.value)
    # three of them fit
    gpu.ttsh_reseed_noalloc(s.ctx, [1, 2, 3], [0, 0, 0], 0.0, 1)
    s.sync()
    assert np.array_equal(s.state(0), kept)
    for i in (1, 2, 3):
        assert np.array_equal(s.state(i), kept)
    s.close()
