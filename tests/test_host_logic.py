"""Host-side logic that needs no GPU: workload definitions, the sweep's chain
map, the algorithmic-byte model used for the roofline, and the binding's
refusal to run without the HIP library."""
import importlib
import math
import sys

import numpy as np
import pytest

from paper_2304_03306_amd import workloads as W


def test_radius_sweep_definition():
    wl = W.radius_sweep()
    assert len(wl.instances) == 64
    radii = sorted({i.radii[0] for i in wl.instances})
    assert len(radii) == 32 and radii[0] == 8.0 and radii[-1] == 80.0
    for i in wl.instances:
        assert abs(i.L - 3.2 * i.radii[0]) < 1e-12
        assert i.L / i.N <= 0.5 + 1e-12
        assert i.N == 128 or i.L / (i.N // 2) > 0.5  # smallest admissible grid
    counts = {N: sum(1 for i in wl.instances if i.N == N) for N in (128, 256, 512)}
    assert counts == {128: 12, 256: 16, 512: 36}
    assert wl.points == 12 * 128 ** 2 + 16 * 256 ** 2 + 36 * 512 ** 2 == 10_682_368


def test_sweep_chain_map():
    src = W.sweep_chain(32)
    assert len(src) == 64
    for j in range(32):
        up, down = 2 * j, 2 * j + 1
        assert src[up] == (2 * (j - 1) if j else up)          # up ramp takes radius j-1
        assert src[down] == (2 * (j + 1) + 1 if j < 31 else down)  # down ramp takes radius j+1
    # every source is on the same ramp as its destination
    assert all(s % 2 == d % 2 for d, s in enumerate(src))


def test_dumbbell_definition():
    wl = W.dumbbells()
    assert len(wl.instances) == 16
    d = [i.centers[1][0] - i.centers[0][0] for i in wl.instances]
    assert abs(d[0] - 40) < 1e-12 and abs(d[-1] - 80) < 1e-12
    assert all(i.N == 1024 and i.L == 256.0 and i.radii == [40.0, 40.0] for i in wl.instances)


def test_uniform_field_is_seeded_and_rounded():
    a = W.uniform_field(3, 16, 0.01, 32)
    b = W.uniform_field(3, 16, 0.01, 32)
    assert np.array_equal(a, b)
    assert np.array_equal(a, a.astype(np.float32).astype(np.float64))
    assert np.abs(a).max() <= 0.01 and a.shape == (2, 16, 16)
    assert not np.array_equal(a, W.uniform_field(4, 16, 0.01, 32))


def test_binary_outside():
    N, L = 32, 32.0
    b = W.binary_outside(N, L, [(0.0, 0.0)], [8.0])
    assert b.dtype == np.uint8
    assert b[N // 2, N // 2] == 0 and b[0, 0] == 1
    assert b[N // 2, N // 2 + 8] == 1  # ||x|| >= R is wall


def test_algorithmic_bytes_model():
    import bench
    # kept modes of the half disk for M = 128
    M = 128
    brute = sum(1 for mx in range(M + 1) for my in range(-M, M + 1) if mx * mx + my * my <= M * M)
    assert bench.kept_modes(512) == brute
    row, col = bench.pass_bytes(512, 8)
    assert abs((row + col) / 512 ** 2 - 26.5) < 1.0  # ~ 28 B/pt with the full rectangle


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_2304_03306_amd import ttsh
    monkeypatch.setattr(ttsh, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(ttsh, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        ttsh.lib()


def test_surrogate_split_and_pair_indexing():
    """Held-out radii take both ramps; pair indices address D[t][i] with the
    successor D[t+1][i] at index + I; the threshold search finds the first
    step above it (NaN counts as above)."""
    import numpy as np
    from paper_2304_03306_amd import surrogate as S
    train, test = S.split_by_radius(32)
    assert test == [2 * j + r for j in (3, 7, 11, 15, 19, 23, 27, 31) for r in (0, 1)]
    assert sorted(train + test) == list(range(64)) and not set(train) & set(test)
    D = np.zeros((5, 4, 2, 2, 3))  # [n_snap][I][Nc][Nc][3]
    idx = S.Trainer.pairs(None, D, [1, 3])
    assert idx.tolist() == [1, 3, 5, 7, 9, 11, 13, 15]
    assert (idx // 4).max() == 3  # every pair's successor (t + 1) exists
    assert S.first_exceeding(np.array([0.01, 0.05, 0.2, 0.01]), 0.1) == 2
    assert S.first_exceeding(np.array([0.01, np.nan]), 0.1) == 1
    assert S.first_exceeding(np.array([0.01, 0.02]), 0.1) == 2


def test_pmc_summary_scaling_and_source_check(tmp_path, monkeypatch):
    """The traffic summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
    by the bytes a known device copy moves per counted byte, averages over
    dispatches, and bench reports it only while the kernel sources hash the
    same."""
    import json
    import bench

    def csv(path, rows):
        with open(path, "w") as f:
            f.write('"Kernel_Name","Counter_Name","Counter_Value"\n')
            for k, c, v in rows:
                f.write(f'"{k}","{c}",{v}\n')
    row = bench.kernel_name("row", 64, 8)
    col = bench.kernel_name("col", 128, 9)
    assert row == "void ttsh::row_multi<float, false, 64, 8>(ttsh::MultiArgs)"
    assert col == "void ttsh::col_multi<float, float, false, 0, 128, 9>(ttsh::MultiArgs)"
    csv(tmp_path / "f.csv", [(row, "FETCH_SIZE", 100.0), (row, "FETCH_SIZE", 300.0), (col, "FETCH_SIZE", 50.0)])
    csv(tmp_path / "w.csv", [(row, "WRITE_SIZE", 40.0), (col, "WRITE_SIZE", 80.0)])
    csv(tmp_path / "cf.csv", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0)])  # 1 MiB read, counted half
    csv(tmp_path / "cw.csv", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)])
    s = bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                            str(tmp_path / "cw.csv"), 1)
    assert s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    assert s["kernels"][row]["bytes"] == 200.0 * 1024 * 2 + 40.0 * 1024
    out = tmp_path / "t.json"
    out.write_text(json.dumps(s))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic(row) == s["kernels"][row]["bytes"]
    assert bench.measured_traffic(col) == s["kernels"][col]["bytes"]
    assert bench.measured_traffic(bench.kernel_name("row", 128, 8)) is None
    s["source_sha256"] = "0" * 64
    out.write_text(json.dumps(s))
    assert bench.measured_traffic(row) is None


def test_philox_known_answers():
    """The Python Philox-4x32-10 against the published known-answer vectors of
    the generator's authors (Salmon et al., SC'11, Random123 test set)."""
    from paper_2304_03306_amd import workloads as W
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        assert tuple(int(w) for w in W.philox4x32_10(ctr, key)) == want


def test_philox_noise_layout_and_range():
    """philox_noise: node (i, j) uses counter (iN + j, instance, 0, 0), word c
    gives component c; values lie in [-amp, amp) and are 24-bit grid values."""
    from paper_2304_03306_amd import workloads as W
    N, amp, seed, inst = 16, 1e-3, (7 << 32) | 5, 3
    z = W.philox_noise(seed, inst, N, amp)
    i, j = 5, 11
    w = W.philox4x32_10((i * N + j, inst, 0, 0), (5, 7))
    for c in range(2):
        assert z[c, i, j] == amp * (2.0 * (int(w[c]) >> 8) * 2.0 ** -24 - 1.0)
    assert z.min() >= -amp and z.max() < amp
    assert not np.array_equal(z, W.philox_noise(seed, inst + 1, N, amp))
    assert not np.array_equal(z, W.philox_noise(seed + 1, inst, N, amp))


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """The tuner cache: the key ignores instance order, a stored choice is
    read back and applied without tuning, a miss tunes and records, and a
    malformed file reads as empty."""
    from paper_2304_03306_amd import tuning, ttsh as T
    monkeypatch.setattr(T, "ttsh_device_arch", lambda: "gfx950:test")
    k1 = tuning.cache_key([512, 128, 512, 256], 32, False, "gfx950:test")
    k2 = tuning.cache_key([256, 512, 128, 512], 32, False, "gfx950:test")
    assert k1 == k2 == "gfx950:test|p32|gw0|1x128,1x256,2x512"
    assert tuning.cache_key([512], 32, True, "a") != tuning.cache_key([512], 64, True, "a")

    class FakeSolver:
        N, precision, gw = [512, 128], 32, False

        def __init__(self):
            self.tuned = 0
            self.applied = None

        def tune(self, n):
            self.tuned += 1
            return (64, 256, 0, 0, 9, 8), 77.5

        def set_tuning(self, cfg):
            self.applied = tuple(cfg)

    path = tmp_path / "cache.json"
    a = FakeSolver()
    cfg, us, hit = tuning.autotune(a, 5, path)
    assert (cfg, us, hit) == ((64, 256, 0, 0, 9, 8), 77.5, False) and a.tuned == 1
    b = FakeSolver()
    cfg, us, hit = tuning.autotune(b, 5, path)
    assert hit and b.tuned == 0 and b.applied == (64, 256, 0, 0, 9, 8) and us == 77.5
    c = FakeSolver()
    tuning.autotune(c, 5, path, retune=True)
    assert c.tuned == 1
    path.write_text("{not json")
    assert tuning.load(path) == {}
    d = FakeSolver()
    _, _, hit = tuning.autotune(d, 5, path)
    assert not hit and d.tuned == 1 and json_keys(path) == [tuning.cache_key(d.N, 32, False, "gfx950:test")]


def json_keys(path):
    import json
    with open(path) as f:
        return sorted(json.load(f))
