"""ctypes binding of the FNO surrogate in libttsh.so (functions of
include/fno.h, same names).  Argument marshalling only; device buffers are
torch tensors, host parameter vectors numpy float32 arrays."""
from __future__ import annotations

import ctypes

import numpy as np

from .ttsh import TTSH_OK, TTSHError, lib as _ttsh_lib

_sig_done = False

FNO_OPT_STAGED_GEMM = 1
FNO_OPT_SPECIALIZED = 2
FNO_OPT_CAPTURE = 3
FNO_OPT_TAIL_PROJ = 4
(FNO_CAP_XB, FNO_CAP_H, FNO_CAP_Z, FNO_CAP_T1, FNO_CAP_G, FNO_CAP_O, FNO_CAP_T2) = range(7)
(FNO_CAP_DZ, FNO_CAP_BT1, FNO_CAP_GG, FNO_CAP_GF, FNO_CAP_BT2, FNO_CAP_DH, FNO_CAP_DHL, FNO_CAP_DY) = range(10, 18)


def lib():
    global _sig_done
    L = _ttsh_lib()
    if not _sig_done:
        vp, i32, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
        sig = {
            "fno_create": ([ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32, i32, i32, i32, u64, vp], ctypes.c_int),
            "fno_num_params": ([vp], ctypes.c_int64),
            "fno_set_params": ([vp, vp], ctypes.c_int),
            "fno_get_params": ([vp, vp], ctypes.c_int),
            "fno_get_grads": ([vp, vp], ctypes.c_int),
            "fno_set_option": ([vp, i32, i32], ctypes.c_int),
            "fno_capture": ([vp, i32, i32, vp, i64], ctypes.c_int),
            "fno_forward": ([vp, vp, vp, i32, i32], ctypes.c_int),
            "fno_forward_ex": ([vp, vp, vp, i64, i32, i32, i32], ctypes.c_int),
            "fno_gather": ([vp, vp, i64, vp, i64, i32, i64, vp, i32], ctypes.c_int),
            "fno_gather_d4": ([vp, vp, i64, vp, i64, i32, i32, vp, vp, i32], ctypes.c_int),
            "fno_perturb": ([vp, vp, i64, i32, i64, f32, u64], ctypes.c_int),
            "fno_sample_errors": ([vp, i64, vp, i64, i32, i64, i32, vp], ctypes.c_int),
            "fno_loss": ([vp, vp, vp, i32, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "fno_loss_ex": ([vp, vp, vp, vp, i64, i32, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "fno_backward": ([vp, i32], ctypes.c_int),
            "fno_adam_step": ([vp, f32, f32, f32, f32], ctypes.c_int),
            "fno_gemm_bf16": ([i32, i32, i32, i32, f32, vp, i64, i64, i64, vp, i64, i64, i64, vp, i64, i64, i64],
                              ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        L.fno_destroy.argtypes = [vp]
        L.fno_destroy.restype = None
        _sig_done = True
    return L


def _check(rc):
    if rc != TTSH_OK:
        raise TTSHError(rc, _ttsh_lib().ttsh_last_error().decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def fno_gemm_bf16(batch, M, N, K, alpha, A, sA, rA, cA, B, sB, rB, cB, C, sC, rC, cC):
    return _check(lib().fno_gemm_bf16(batch, M, N, K, alpha, _ptr(A), sA, rA, cA, _ptr(B), sB, rB, cB,
                                      _ptr(C), sC, rC, cC))


def fno_sample_errors(y, ys, t, ts, nch, npix, batch):
    """Per-sample relative L2 errors (numpy float64 [batch])."""
    out = np.empty(batch, dtype=np.float64)
    _check(lib().fno_sample_errors(_ptr(y), ys, _ptr(t), ts, nch, npix, batch,
                                   out.ctypes.data_as(ctypes.c_void_p)))
    return out


class FNO:
    """One network on the GPU (fno_create ... fno_destroy)."""

    def __init__(self, width=32, modes=16, layers=4, cin=3, cout=2, hidden=128, H=128, W=128,
                 max_batch=256, seed=0, stream=None):
        self.cfg = dict(width=width, modes=modes, layers=layers, cin=cin, cout=cout, hidden=hidden, H=H, W=W)
        self.ctx = ctypes.c_void_p()
        _check(lib().fno_create(ctypes.byref(self.ctx), width, modes, layers, cin, cout, hidden, H, W,
                                max_batch, seed, ctypes.c_void_p(stream or 0)))
        self.n = int(lib().fno_num_params(self.ctx))

    def close(self):
        if self.ctx:
            lib().fno_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p: np.ndarray):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.n
        _check(lib().fno_set_params(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))

    def params(self) -> np.ndarray:
        a = np.empty(self.n, dtype=np.float32)
        _check(lib().fno_get_params(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def grads(self) -> np.ndarray:
        a = np.empty(self.n, dtype=np.float32)
        _check(lib().fno_get_grads(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def capture(self, what: int, layer: int, n: int) -> np.ndarray:
        """The first n captured BF16 values of an item (FNO_CAP_*), float64."""
        out = np.empty(int(n), dtype=np.float32)
        _check(lib().fno_capture(self.ctx, int(what), int(layer), out.ctypes.data_as(ctypes.c_void_p), int(n)))
        return out.astype(np.float64)

    def set_option(self, option: int, value: int):
        _check(lib().fno_set_option(self.ctx, int(option), int(value)))

    def forward(self, x, y, train=False):
        _check(lib().fno_forward(self.ctx, _ptr(x), _ptr(y), int(x.shape[0]), int(bool(train))))

    def forward_ex(self, x, y, y_pix_stride, residual, batch, train=False):
        """y may be a tensor or a raw device address (int) inside x."""
        yp = ctypes.c_void_p(y) if isinstance(y, int) else _ptr(y)
        _check(lib().fno_forward_ex(self.ctx, _ptr(x), yp, int(y_pix_stride), int(bool(residual)), int(batch),
                                    int(bool(train))))

    def perturb(self, x, pix_stride, nch, npix, amp, seed):
        _check(lib().fno_perturb(self.ctx, _ptr(x), int(pix_stride), int(nch), int(npix), float(amp), int(seed)))

    def gather_d4(self, dst, dst_ch, src, src_ch, nch, n_side, idx, sym):
        """gather of square samples with the D4 symmetry sym[s] (0..7) applied
        to sample s (fno_gather_d4)."""
        ix = np.ascontiguousarray(idx, dtype=np.int64)
        sy = np.ascontiguousarray(sym, dtype=np.int32)
        npix = n_side * n_side
        if ix.size != sy.size:
            raise ValueError("one symmetry element per sample")
        if ix.size and int(ix.max()) * npix * src_ch + npix * src_ch > src.numel():
            raise ValueError("sample index beyond the source")
        _check(lib().fno_gather_d4(self.ctx, _ptr(dst), int(dst_ch), _ptr(src), int(src_ch), int(nch), int(n_side),
                                   ix.ctypes.data_as(ctypes.c_void_p), sy.ctypes.data_as(ctypes.c_void_p),
                                   int(ix.size)))

    def gather(self, dst, dst_ch, src, src_ch, nch, npix, idx):
        """Copy samples idx (host int64 indices) of src into dst."""
        ix = np.ascontiguousarray(idx, dtype=np.int64)
        if ix.size and int(ix.max()) * npix * src_ch + npix * src_ch > src.numel():
            raise ValueError("sample index beyond the source")
        _check(lib().fno_gather(self.ctx, _ptr(dst), int(dst_ch), _ptr(src), int(src_ch), int(nch), int(npix),
                                ix.ctypes.data_as(ctypes.c_void_p), int(ix.size)))

    def loss(self, y, t):
        out = ctypes.c_double()
        _check(lib().fno_loss(self.ctx, _ptr(y), _ptr(t), int(y.shape[0]), ctypes.byref(out)))
        return out.value

    def loss_ex(self, y, t, ref, ref_stride, batch):
        out = ctypes.c_double()
        _check(lib().fno_loss_ex(self.ctx, _ptr(y), _ptr(t), _ptr(ref), int(ref_stride), int(batch),
                                 ctypes.byref(out)))
        return out.value

    def backward(self, batch):
        _check(lib().fno_backward(self.ctx, int(batch)))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().fno_adam_step(self.ctx, lr, beta1, beta2, eps))


def flatten_params(p: dict, layers: int) -> np.ndarray:
    """Oracle parameter dict -> the library's flat float32 vector."""
    parts = [p["P_w"], p["P_b"]]
    for l in range(layers):
        parts += [p[f"R{l}"].real, p[f"R{l}"].imag, p[f"W{l}"], p[f"b{l}"]]
    parts += [p["Q1_w"], p["Q1_b"], p["Q2_w"], p["Q2_b"]]
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts]).astype(np.float32)


def unflatten(vec: np.ndarray, like: dict, layers: int) -> dict:
    """Flat vector -> dict shaped like the oracle's parameters (R complex)."""
    out, o = {}, 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        a = vec[o:o + n].reshape(shape).astype(np.float64)
        o += n
        return a

    out["P_w"] = take(like["P_w"].shape)
    out["P_b"] = take(like["P_b"].shape)
    for l in range(layers):
        re = take(like[f"R{l}"].shape)
        im = take(like[f"R{l}"].shape)
        out[f"R{l}"] = re + 1j * im
        out[f"W{l}"] = take(like[f"W{l}"].shape)
        out[f"b{l}"] = take(like[f"b{l}"].shape)
    for k in ("Q1_w", "Q1_b", "Q2_w", "Q2_b"):
        out[k] = take(like[k].shape)
    return out


def main(argv=None):
    """Time the network on random inputs: inference (residual, in place) and
    one training step (forward, loss, backward, Adam), HIP-synchronised."""
    import argparse
    import time

    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, default=16)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--iters", type=int, default=5)
    ap.add_argument("--no-train", action="store_true")
    a = ap.parse_args(argv)
    B, n = a.batch, a.size
    net = FNO(width=a.width, modes=a.modes, layers=a.layers, cin=3, cout=2, hidden=a.hidden, H=n, W=n,
              max_batch=B, seed=0)
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(B, n, n, 3, device="cuda", generator=gen)
    t = torch.randn(B, n, n, 2, device="cuda", generator=gen)
    y = torch.empty(B, n, n, 2, device="cuda")
    net.forward_ex(x, y, 2, True, B)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(a.iters):
        net.forward_ex(x, y, 2, True, B)
    torch.cuda.synchronize()
    inf = (time.time() - t0) / a.iters
    out = {"batch": B, "size": n, "inference_ms": inf * 1e3}
    if not a.no_train:
        t0 = time.time()
        for _ in range(a.iters):
            net.forward_ex(x, y, 2, True, B, train=True)
            net.loss(y, t)
            net.backward(B)
            net.adam_step(1e-4)
        torch.cuda.synchronize()
        out["train_step_ms"] = (time.time() - t0) / a.iters * 1e3
    print(out, flush=True)
    return out


if __name__ == "__main__":
    main()
