"""ctypes binding of libttsh.so (functions of include/ttsh.h, same names).

Argument marshalling only: every step of the computation runs in the HIP
library.  Host buffers are numpy arrays (passed with TTSH_HOST); device
buffers are torch tensors on a ROCm device (passed with TTSH_DEVICE by their
data pointer).  A missing library raises at import of this module's functions;
there is no fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().with_name("libttsh.so")

TTSH_OK, TTSH_EINVAL, TTSH_EUNSUPPORTED, TTSH_EHIP, TTSH_ENONFINITE, TTSH_ENOMEM = 0, -1, -2, -3, -4, -5
TTSH_HOST, TTSH_DEVICE = 0, 1
TTSH_IFEULER, TTSH_ETD1, TTSH_IMEX, TTSH_ETDRK2, TTSH_ETDRK4 = 0, 1, 2, 3, 4
TTSH_FP32, TTSH_FP64, TTSH_FP32_STATE64 = 32, 64, 96
TTSH_OPT_GRAPH_STEPS, TTSH_OPT_BLOCK, TTSH_OPT_GUARD, TTSH_OPT_SPLIT, TTSH_OPT_GUARD_EVERY = 1, 2, 4, 8, 16
TTSH_OPT_GROUPS = 17
TUNING_INTS = 7  # row size, column size, row split, column split, row schedule, column schedule, groups
SCHEMES = {"ifeuler": TTSH_IFEULER, "etd1": TTSH_ETD1, "imex": TTSH_IMEX, "etdrk2": TTSH_ETDRK2,
           "etdrk4": TTSH_ETDRK4}


class TTSHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ttsh error {code}: {msg}")
        self.code = code


class ttsh_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("alpha", "beta", "gamma0", "gamma2", "lambda0", "lambda1", "gamma_v", "gamma_w", "dt")] + \
               [("scheme", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libttsh.so (built in-tree by paper_2304_03306_amd.build)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_03306_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "ttsh_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ttsh_params), i32, vp],
            "ttsh_set_mask": [vp, i32, dp, i32],
            "ttsh_get_mask": [vp, i32, dp, i32],
            "ttsh_mask_tanh": [vp, i32, i32, dp, dp, dp, ctypes.c_double],
            "ttsh_mask_from_binary": [vp, i32, dp, i32],
            "ttsh_set_field": [vp, i32, dp, i32],
            "ttsh_get_field": [vp, i32, dp, dp, i32],
            "ttsh_get_field_coarse": [vp, i32, i32, dp, i64],
            "ttsh_set_field_coarse": [vp, i32, i32, dp, i64],
            "ttsh_project_coarse": [vp, i32, dp, i64, i32, dp],
            "ttsh_order": [vp, i32, ctypes.c_double, ctypes.c_double, dp],
            "ttsh_order_dumbbell": [vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp],
            "ttsh_vortices": [vp, i32, ctypes.c_double, ctypes.c_double, dp],
            "ttsh_lyap_qr": [vp, i32, vp, i32, ctypes.c_double, dp],
            "ttsh_psd_accumulate": [vp, i32, i32, dp, ctypes.c_double, vp],
            "ttsh_psd_finish": [vp, i32, i32, vp, dp],
            "ttsh_set_state": [vp, i32, dp, i32],
            "ttsh_get_state": [vp, i32, dp, i32],
            "ttsh_step": [vp, i64],
            "ttsh_reseed": [vp, i32, dp, dp, ctypes.c_double, ctypes.c_uint64],
            "ttsh_reseed_field": [vp, i32, dp, dp, dp, i32],
            "ttsh_reseed_noalloc": [vp, i32, dp, dp, ctypes.c_double, ctypes.c_uint64],
            "ttsh_norms": [vp, i32, dp],
            "ttsh_sync": [vp],
            "ttsh_set_option": [vp, i32, i64],
            "ttsh_fft2": [dp, dp, i32, i32, i32, i32],
            "ttsh_pass_times": [vp, i64, dp],
            "ttsh_tune": [vp, i64, dp, dp],
            "ttsh_get_tuning": [vp, dp],
            "ttsh_set_tuning": [vp, dp],
            "ttsh_device_arch": [dp, i32],
            "ttsh_num_classes": [vp, dp],
            "ttsh_stream_bench": [i32, i32, i64, i32, i32, vp, dp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ttsh_destroy.argtypes = [vp]
        L.ttsh_destroy.restype = None
        L.ttsh_last_error.argtypes = []
        L.ttsh_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != TTSH_OK:
        raise TTSHError(rc, lib().ttsh_last_error().decode())
    return rc


def _buf(x, dtype):
    """(pointer, where, keepalive) of a numpy array (host) or torch tensor (device)."""
    if x is None:
        return None, TTSH_HOST, None
    if isinstance(x, np.ndarray):
        a = np.ascontiguousarray(x, dtype=dtype)
        return a.ctypes.data_as(ctypes.c_void_p), TTSH_HOST, a
    # torch tensor on the GPU
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("device buffers must be contiguous GPU tensors")
    return ctypes.c_void_p(x.data_ptr()), TTSH_DEVICE, x


def make_params(p) -> ttsh_params:
    """ttsh_params from any object with the coefficient attributes."""
    scheme = getattr(p, "scheme", "ifeuler")
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    return ttsh_params(p.alpha, p.beta, p.gamma0, p.gamma2, p.lambda0, p.lambda1,
                       p.gamma_v, p.gamma_w, p.dt, int(scheme))


# ---- functions of the C interface ------------------------------------------------
def ttsh_create(N, L, params, precision=TTSH_FP32, stream=None):
    n = len(N)
    Na = (ctypes.c_int * n)(*[int(v) for v in N])
    La = (ctypes.c_double * n)(*[float(v) for v in L])
    prm = params if isinstance(params, ttsh_params) else make_params(params)
    ctx = ctypes.c_void_p()
    _check(lib().ttsh_create(ctypes.byref(ctx), n, Na, La, ctypes.byref(prm), int(precision),
                             ctypes.c_void_p(stream or 0)))
    return ctx


def ttsh_destroy(ctx):
    lib().ttsh_destroy(ctx)


def ttsh_set_mask(ctx, inst, K):
    p, w, keep = _buf(K, np.float64)
    return _check(lib().ttsh_set_mask(ctx, inst, p, w))


def ttsh_get_mask(ctx, inst, out):
    p, w, keep = _buf(out, np.float64)
    _check(lib().ttsh_get_mask(ctx, inst, p, w))
    return out


def ttsh_mask_tanh(ctx, inst, centers, radii, xi):
    n = len(radii)
    cx = np.ascontiguousarray([c[0] for c in centers], dtype=np.float64)
    cy = np.ascontiguousarray([c[1] for c in centers], dtype=np.float64)
    R = np.ascontiguousarray(radii, dtype=np.float64)
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    return _check(lib().ttsh_mask_tanh(ctx, inst, n, f(cx), f(cy), f(R), float(xi)))


def ttsh_mask_from_binary(ctx, inst, K_naive):
    p, w, keep = _buf(K_naive, np.uint8)
    return _check(lib().ttsh_mask_from_binary(ctx, inst, p, w))


def ttsh_set_field(ctx, inst, v):
    p, w, keep = _buf(v, np.float64)
    return _check(lib().ttsh_set_field(ctx, inst, p, w))


def ttsh_get_field(ctx, inst, v_out, omega_out=None):
    p, w, keep = _buf(v_out, np.float64)
    q, w2, keep2 = _buf(omega_out, np.float64)
    if omega_out is not None and w2 != w:
        raise ValueError("v and omega must both be host or both be device buffers")
    _check(lib().ttsh_get_field(ctx, inst, p, q, w))
    return v_out, omega_out


def ttsh_get_field_coarse(ctx, inst, Nc, out, pix_stride=2):
    """out: float32 GPU tensor holding at least Nc*Nc*pix_stride values;
    component c of node (i, j) lands at flat index (i*Nc + j)*pix_stride + c."""
    if not out.is_cuda or out.dtype.itemsize != 4:
        raise ValueError("out must be a float32 GPU tensor")
    if out.numel() < (Nc * Nc - 1) * pix_stride + 2:
        raise ValueError("out too small")
    return _check(lib().ttsh_get_field_coarse(ctx, int(inst), int(Nc), ctypes.c_void_p(out.data_ptr()),
                                              int(pix_stride)))


def ttsh_order(ctx, inst, center=(0.0, 0.0)):
    """(Psi about center, Psi_2 split at x = center[0])."""
    out = (ctypes.c_double * 2)()
    _check(lib().ttsh_order(ctx, int(inst), float(center[0]), float(center[1]), ctypes.cast(out, ctypes.c_void_p)))
    return out[0], out[1]

def ttsh_order_dumbbell(ctx, inst, D, center=(0.0, 0.0)):
    """Psi_2 over the disks of radius D/2 about center -+ (D/2, 0)."""
    out = ctypes.c_double()
    _check(lib().ttsh_order_dumbbell(ctx, int(inst), float(center[0]), float(center[1]), float(D),
                                     ctypes.cast(ctypes.pointer(out), ctypes.c_void_p)))
    return out.value

def ttsh_lyap_qr(ctx, base, pert, eps):
    """log R_vv of the re-orthonormalised deviations of instances pert from
    base (see include/ttsh.h); the perturbed states are rewritten."""
    pert = [int(x) for x in pert]
    idx = (ctypes.c_int * max(1, len(pert)))(*pert)
    out = (ctypes.c_double * max(1, len(pert)))()
    _check(lib().ttsh_lyap_qr(ctx, int(base), ctypes.cast(idx, ctypes.c_void_p), len(pert), float(eps),
                              ctypes.cast(out, ctypes.c_void_p)))
    return np.array(out[: len(pert)], dtype=np.float64)

def psd_buffer_len(N, nf):
    """Float64 entries of a PSD accumulator for grid size N and nf
    frequencies (see include/ttsh.h: nf * 2 * (N/4+1) * (N/2+2) complex)."""
    return 2 * nf * 2 * (N // 4 + 1) * (N // 2 + 2)


def ttsh_psd_accumulate(ctx, inst, freqs, t, acc):
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    _check(lib().ttsh_psd_accumulate(ctx, int(inst), len(f), f.ctypes.data_as(ctypes.c_void_p), float(t),
                                     _dev_addr(acc)))


def ttsh_psd_finish(ctx, N, nf, acc):
    out = np.zeros(int(nf), dtype=np.float64)
    _check(lib().ttsh_psd_finish(ctx, int(N), int(nf), _dev_addr(acc), out.ctypes.data_as(ctypes.c_void_p)))
    return out

def ttsh_vortices(ctx, inst, kmax=0.5, vmin=0.0):
    """(vortex centres, saddles) of instance inst, see include/ttsh.h."""
    out = (ctypes.c_int * 2)()
    _check(lib().ttsh_vortices(ctx, int(inst), float(kmax), float(vmin), ctypes.cast(out, ctypes.c_void_p)))
    return int(out[0]), int(out[1])


def _dev_addr(x):
    return ctypes.c_void_p(x if isinstance(x, int) else x.data_ptr())


def ttsh_set_field_coarse(ctx, inst, Nc, v, pix_stride=2):
    """v: float32 GPU tensor (or device address) laid out as for
    ttsh_get_field_coarse."""
    return _check(lib().ttsh_set_field_coarse(ctx, int(inst), int(Nc), _dev_addr(v), int(pix_stride)))


def ttsh_project_coarse(ctx, N, v, pix_stride, batch, norms=False):
    """Project `batch` float32 fields in place; returns [batch][2] norms if asked."""
    out = np.empty((batch, 2), dtype=np.float64) if norms else None
    _check(lib().ttsh_project_coarse(ctx, int(N), _dev_addr(v), int(pix_stride), int(batch),
                                     out.ctypes.data_as(ctypes.c_void_p) if norms else None))
    return out


def ttsh_set_state(ctx, inst, vhat):
    p, w, keep = _buf(vhat, np.complex128)
    return _check(lib().ttsh_set_state(ctx, inst, p, w))


def ttsh_get_state(ctx, inst, out):
    p, w, keep = _buf(out, np.complex128)
    _check(lib().ttsh_get_state(ctx, inst, p, w))
    return out


def ttsh_step(ctx, nsteps):
    return _check(lib().ttsh_step(ctx, int(nsteps)))


def _index_lists(dst, src):
    n = len(dst)
    if len(src) != n:
        raise ValueError("dst and src must have the same length")
    d = (ctypes.c_int * n)(*[int(v) for v in dst])
    s = (ctypes.c_int * n)(*[int(v) for v in src])
    return n, d, s


def ttsh_reseed(ctx, dst, src, noise_amp=0.0, seed=0):
    n, d, s = _index_lists(dst, src)
    return _check(lib().ttsh_reseed(ctx, n, ctypes.cast(d, ctypes.c_void_p), ctypes.cast(s, ctypes.c_void_p),
                                    float(noise_amp), int(seed) & 0xFFFFFFFFFFFFFFFF))


def ttsh_reseed_noalloc(ctx, dst, src, noise_amp=0.0, seed=0):
    n, d, s = _index_lists(dst, src)
    return _check(lib().ttsh_reseed_noalloc(ctx, n, ctypes.cast(d, ctypes.c_void_p),
                                            ctypes.cast(s, ctypes.c_void_p), float(noise_amp),
                                            int(seed) & 0xFFFFFFFFFFFFFFFF))


def ttsh_reseed_field(ctx, dst, src, noise=None):
    n, d, s = _index_lists(dst, src)
    p, w, keep = _buf(noise, np.float64)
    return _check(lib().ttsh_reseed_field(ctx, n, ctypes.cast(d, ctypes.c_void_p),
                                          ctypes.cast(s, ctypes.c_void_p), p, w))


def ttsh_norms(ctx, inst):
    out = (ctypes.c_double * 4)()
    _check(lib().ttsh_norms(ctx, inst, ctypes.cast(out, ctypes.c_void_p)))
    return list(out)


def ttsh_sync(ctx):
    return _check(lib().ttsh_sync(ctx))


def ttsh_set_option(ctx, key, value):
    return _check(lib().ttsh_set_option(ctx, int(key), int(value)))


def ttsh_fft2(inp, out, N, batch, inverse, precision):
    """Device tensors (complex128 viewed as float64 pairs)."""
    return _check(lib().ttsh_fft2(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  int(N), int(batch), int(bool(inverse)), int(precision)))


def ttsh_num_classes(ctx):
    n = lib().ttsh_num_classes(ctx, None)
    if n < 0:
        _check(n)
    sizes = (ctypes.c_int * max(n, 1))()
    lib().ttsh_num_classes(ctx, ctypes.cast(sizes, ctypes.c_void_p))
    return list(sizes)[:n]


def ttsh_pass_times(ctx, nsteps):
    """(row_us, col_us): mean durations of the two launches of a step, from
    HIP events."""
    out = (ctypes.c_double * 2)()
    _check(lib().ttsh_pass_times(ctx, int(nsteps), ctypes.cast(out, ctypes.c_void_p)))
    return out[0], out[1]


def ttsh_stream_bench(reads, writes, elems, blocks, reps, buf):
    """Mean microseconds per launch of the streaming probe (reads, writes
    arrays of `elems` 16-byte elements) on the device buffer `buf` (a torch
    tensor or a device address) of at least (reads + max(writes, 1)) * elems
    * 16 bytes."""
    need = (reads + max(writes, 1)) * int(elems) * 16
    if hasattr(buf, "data_ptr"):
        if buf.numel() * buf.element_size() < need:
            raise ValueError("stream buffer too small")
        ptr = buf.data_ptr()
    else:
        ptr = int(buf)
    out = ctypes.c_double()
    _check(lib().ttsh_stream_bench(int(reads), int(writes), int(elems), int(blocks), int(reps),
                                   ctypes.c_void_p(ptr), ctypes.byref(out)))
    return out.value


def ttsh_tune(ctx, nsteps):
    """Pick the fastest launch configuration; returns ((row_size, col_size,
    row_split, col_split, row_schedule, col_schedule, groups), us_per_step)."""
    cfg = (ctypes.c_int * TUNING_INTS)()
    us = ctypes.c_double()
    _check(lib().ttsh_tune(ctx, int(nsteps), ctypes.cast(cfg, ctypes.c_void_p),
                           ctypes.cast(ctypes.byref(us), ctypes.c_void_p)))
    return tuple(cfg), us.value


def ttsh_get_tuning(ctx):
    cfg = (ctypes.c_int * TUNING_INTS)()
    _check(lib().ttsh_get_tuning(ctx, ctypes.cast(cfg, ctypes.c_void_p)))
    return tuple(cfg)


def ttsh_set_tuning(ctx, cfg):
    """Set a configuration of TUNING_INTS ints; one of 6 (without the group
    count) means one group."""
    cfg = [int(v) for v in cfg]
    if len(cfg) == TUNING_INTS - 1:
        cfg.append(1)
    if len(cfg) != TUNING_INTS:
        raise ValueError(f"a tuning is {TUNING_INTS} ints")
    arr = (ctypes.c_int * TUNING_INTS)(*cfg)
    return _check(lib().ttsh_set_tuning(ctx, ctypes.cast(arr, ctypes.c_void_p)))


def ttsh_device_arch():
    buf = ctypes.create_string_buffer(128)
    _check(lib().ttsh_device_arch(ctypes.cast(buf, ctypes.c_void_p), 128))
    return buf.value.decode()


def ttsh_last_error() -> str:
    return lib().ttsh_last_error().decode()


# ---- convenience wrapper ------------------------------------------------------------
class Solver:
    """Owns one context.  N, L: per-instance lists; params: coefficients object."""

    def __init__(self, N, L, params, precision=TTSH_FP32, stream=None):
        self.N = [int(n) for n in N]
        self.L = [float(x) for x in L]
        self.precision = int(precision)
        self.gw = float(getattr(params, "gamma_w", 0.0)) != 0.0
        self.ctx = ttsh_create(self.N, self.L, params, precision, stream)

    def close(self):
        if self.ctx:
            ttsh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mask_tanh(self, inst, centers, radii, xi):
        ttsh_mask_tanh(self.ctx, inst, centers, radii, xi)

    def mask_from_binary(self, inst, K_naive):
        ttsh_mask_from_binary(self.ctx, inst, K_naive)

    def set_mask(self, inst, K):
        ttsh_set_mask(self.ctx, inst, K)

    def mask(self, inst):
        n = self.N[inst]
        return ttsh_get_mask(self.ctx, inst, np.empty((n, n)))

    def set_field(self, inst, v):
        ttsh_set_field(self.ctx, inst, v)

    def field(self, inst, omega=False):
        n = self.N[inst]
        v = np.empty((2, n, n))
        w = np.empty((n, n)) if omega else None
        ttsh_get_field(self.ctx, inst, v, w)
        return (v, w) if omega else v

    def order(self, inst, center=(0.0, 0.0)):
        return ttsh_order(self.ctx, inst, center)

    def order_dumbbell(self, inst, D, center=(0.0, 0.0)):
        return ttsh_order_dumbbell(self.ctx, inst, D, center)

    def lyap_qr(self, base, pert, eps):
        return ttsh_lyap_qr(self.ctx, base, pert, eps)

    def psd_accumulate(self, inst, freqs, t, acc):
        ttsh_psd_accumulate(self.ctx, inst, freqs, t, acc)

    def psd_finish(self, N, nf, acc):
        return ttsh_psd_finish(self.ctx, N, nf, acc)

    def vortices(self, inst, kmax=0.5, vmin=0.0):
        return ttsh_vortices(self.ctx, inst, kmax, vmin)

    def field_coarse(self, inst, Nc, out, pix_stride=2):
        ttsh_get_field_coarse(self.ctx, inst, Nc, out, pix_stride)

    def set_field_coarse(self, inst, Nc, v, pix_stride=2):
        ttsh_set_field_coarse(self.ctx, inst, Nc, v, pix_stride)

    def project_coarse(self, N, v, pix_stride, batch, norms=False):
        return ttsh_project_coarse(self.ctx, N, v, pix_stride, batch, norms)

    def state(self, inst):
        M = self.N[inst] // 4
        return ttsh_get_state(self.ctx, inst, np.empty((2, 2 * M + 1, M + 1), dtype=np.complex128))

    def set_state(self, inst, vhat):
        ttsh_set_state(self.ctx, inst, vhat)

    def step(self, n):
        ttsh_step(self.ctx, n)

    def sync(self):
        ttsh_sync(self.ctx)

    def norms(self, inst):
        return ttsh_norms(self.ctx, inst)

    def option(self, key, value):
        ttsh_set_option(self.ctx, key, value)

    def reseed(self, dst, src, noise_amp=0.0, seed=0):
        """Continuation with device-drawn (Philox) noise of amplitude noise_amp."""
        ttsh_reseed(self.ctx, dst, src, noise_amp, seed)

    def reseed_field(self, dst, src, noise=None):
        """Continuation with caller-drawn noise fields ([n][2][N][N] or flat)."""
        ttsh_reseed_field(self.ctx, dst, src, noise)

    def tune(self, nsteps=20):
        return ttsh_tune(self.ctx, nsteps)

    def get_tuning(self):
        return ttsh_get_tuning(self.ctx)

    def set_tuning(self, cfg):
        ttsh_set_tuning(self.ctx, cfg)

    def pass_times(self, nsteps=50):
        return ttsh_pass_times(self.ctx, nsteps)
