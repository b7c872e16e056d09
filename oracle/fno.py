"""FP64 CPU oracle of the Fourier-neural-operator surrogate (test
infrastructure only).

Architecture (Fourier neural operator, Li et al., ICLR 2021): per-point lift
P: C_in -> C; L Fourier layers
    h <- act( S_l(h) + h W_l + b_l ),   act = exact GELU except after the last layer,
    S_l(h) = irfft2( pad( R_l . trunc(rfft2(h)) ) ),
with the retained modes k_x = 0..m-1 (half spectrum) and k_y = -m..m-1, and
R_l a complex C x C matrix per retained mode; then the per-point projection
Q: C -> C_h -> GELU -> C_out.  Fields are channels-last [B][H][W][C];
rfft2/irfft2 are numpy's unnormalised forward / 1/(HW) inverse transforms.

The backward pass is written out by hand (no automatic differentiation).
For a complex intermediate z the gradient carried is dl/dRe z + i dl/dIm z.
Its pieces:
    s = irfft2(pad(G)):   g_G[ky,kx] = w_kx/(HW) rfft2(g_s)[ky,kx],  w_0 = 1, w_kx = 2
    G = F R:              g_F = g_G R^H,   g_R = F^H g_G   (per mode, summed over batch)
    F = trunc(rfft2(h)):  g_h = Re( sum over retained modes of g_F e^{+i k.x} )
The tests check it against central finite differences and the adjoint identity.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf


@dataclasses.dataclass
class Config:
    H: int = 128
    W: int = 128
    cin: int = 3
    cout: int = 2
    width: int = 32
    modes: int = 16
    layers: int = 4
    hidden: int = 128


def retained_rows(cfg: Config) -> np.ndarray:
    """FFT-order row indices of k_y = 0..m-1, -m..-1 (2m rows)."""
    m = cfg.modes
    return np.concatenate([np.arange(m), np.arange(cfg.H - m, cfg.H)])


def init_params(cfg: Config, seed: int = 0) -> dict:
    """Random parameters (the layout the library uses, in FP64)."""
    rng = np.random.default_rng(seed)
    C, m = cfg.width, cfg.modes
    p = {
        "P_w": rng.standard_normal((cfg.cin, C)) / math.sqrt(cfg.cin),
        "P_b": np.zeros(C),
        "Q1_w": rng.standard_normal((C, cfg.hidden)) / math.sqrt(C),
        "Q1_b": np.zeros(cfg.hidden),
        "Q2_w": rng.standard_normal((cfg.hidden, cfg.cout)) / math.sqrt(cfg.hidden),
        "Q2_b": np.zeros(cfg.cout),
    }
    scale = 1.0 / (C * C)
    for l in range(cfg.layers):
        p[f"R{l}"] = scale * (rng.uniform(0, 1, (2 * m, m, C, C)) + 1j * rng.uniform(0, 1, (2 * m, m, C, C)))
        p[f"W{l}"] = rng.standard_normal((C, C)) / math.sqrt(C)
        p[f"b{l}"] = np.zeros(C)
    return p


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


# ---- spectral convolution and its adjoints -------------------------------------------
def spectral_forward(h: np.ndarray, R: np.ndarray, cfg: Config):
    """h [B,H,W,C] -> (s [B,H,W,C], F [B,2m,m,C]) with F the retained modes."""
    m = cfg.modes
    rows = retained_rows(cfg)
    Hh = np.fft.rfft2(h, axes=(1, 2))
    F = Hh[:, rows, :m, :]
    G = np.einsum("bykc,ykco->byko", F, R)
    full = np.zeros((h.shape[0], cfg.H, cfg.W // 2 + 1, R.shape[-1]), dtype=np.complex128)
    full[:, rows, :m, :] = G
    s = np.fft.irfft2(full, s=(cfg.H, cfg.W), axes=(1, 2))
    return s, F


def spectral_backward(g_s: np.ndarray, F: np.ndarray, R: np.ndarray, cfg: Config):
    """Gradients (g_h, g_R) of the spectral convolution given g_s = dl/ds."""
    m = cfg.modes
    rows = retained_rows(cfg)
    HW = cfg.H * cfg.W
    w = np.full(m, 2.0)
    w[0] = 1.0
    g_G = np.fft.rfft2(g_s, axes=(1, 2))[:, rows, :m, :] * (w[None, None, :, None] / HW)
    g_F = np.einsum("byko,ykco->bykc", g_G, np.conj(R))
    g_R = np.einsum("bykc,byko->ykco", np.conj(F), g_G)
    full = np.zeros((g_s.shape[0], cfg.H, cfg.W, F.shape[-1]), dtype=np.complex128)
    full[:, rows, :m, :] = g_F
    g_h = np.real(np.fft.ifft2(full, axes=(1, 2))) * HW
    return g_h, g_R


# ---- network -----------------------------------------------------------------------------
def forward(params: dict, x: np.ndarray, cfg: Config, keep: bool = False):
    """x [B,H,W,cin] -> y [B,H,W,cout] (and the saved activations)."""
    cache = {"x": x}
    h = x @ params["P_w"] + params["P_b"]
    for l in range(cfg.layers):
        s, F = spectral_forward(h, params[f"R{l}"], cfg)
        z = s + h @ params[f"W{l}"] + params[f"b{l}"]
        cache[f"h{l}"], cache[f"F{l}"], cache[f"z{l}"] = h, F, z
        h = gelu(z) if l < cfg.layers - 1 else z
    u = h @ params["Q1_w"] + params["Q1_b"]
    a = gelu(u)
    y = a @ params["Q2_w"] + params["Q2_b"]
    cache["h_last"], cache["u"], cache["a"] = h, u, a
    return (y, cache) if keep else y


def rel_l2_loss(y: np.ndarray, t: np.ndarray):
    """Mean over samples of ||y - t||_2 / ||t||_2, and its gradient dl/dy."""
    B = y.shape[0]
    d = (y - t).reshape(B, -1)
    num = np.sqrt(np.sum(d * d, axis=1))
    den = np.sqrt(np.sum(t.reshape(B, -1) ** 2, axis=1))
    loss = float(np.mean(num / den))
    g = (d / (num * den)[:, None] / B).reshape(y.shape)
    return loss, g


def backward(params: dict, cache: dict, g_y: np.ndarray, cfg: Config) -> dict:
    """Hand-written reverse pass; returns dl/dparam for every parameter
    (complex R gradients as dl/dRe + i dl/dIm)."""
    grads = {}
    a, u, h = cache["a"], cache["u"], cache["h_last"]
    flat = lambda t: t.reshape(-1, t.shape[-1])
    grads["Q2_w"] = flat(a).T @ flat(g_y)
    grads["Q2_b"] = flat(g_y).sum(axis=0)
    g_u = (g_y @ params["Q2_w"].T) * gelu_grad(u)
    grads["Q1_w"] = flat(h).T @ flat(g_u)
    grads["Q1_b"] = flat(g_u).sum(axis=0)
    g_h = g_u @ params["Q1_w"].T
    for l in reversed(range(cfg.layers)):
        z, hl, F = cache[f"z{l}"], cache[f"h{l}"], cache[f"F{l}"]
        g_z = g_h * gelu_grad(z) if l < cfg.layers - 1 else g_h
        grads[f"W{l}"] = flat(hl).T @ flat(g_z)
        grads[f"b{l}"] = flat(g_z).sum(axis=0)
        g_hs, g_R = spectral_backward(g_z, F, params[f"R{l}"], cfg)
        grads[f"R{l}"] = g_R
        g_h = g_z @ params[f"W{l}"].T + g_hs
    x = cache["x"]
    grads["P_w"] = flat(x).T @ flat(g_h)
    grads["P_b"] = flat(g_h).sum(axis=0)
    return grads


# ---- optimiser ------------------------------------------------------------------------------
def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015) on real arrays; returns
    (theta, m, v).  t counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---- data: coarsening a solver state --------------------------------------------------------
def coarsen(vhat_full: np.ndarray, Nc: int) -> np.ndarray:
    """Real field on an Nc x Nc grid from a unitary spectrum on a finer grid by
    keeping the modes m_x^2 + m_y^2 <= (Nc/4)^2 (the coarse grid's 1/2-rule
    disk) and transforming back: returns [2][Nc][Nc]."""
    N = vhat_full.shape[-1]
    Mc = Nc // 4
    m = np.fft.fftfreq(N, 1.0 / N).round().astype(int)
    mc = np.fft.fftfreq(Nc, 1.0 / Nc).round().astype(int)
    out = np.zeros(vhat_full.shape[:-2] + (Nc, Nc), dtype=np.complex128)
    for iy, my in enumerate(mc):
        for ix, mx in enumerate(mc):
            if mx * mx + my * my <= Mc * Mc:
                out[..., iy, ix] = vhat_full[..., my % N, mx % N]
    # unitary on both grids: coefficients scale by Nc/N
    return np.fft.ifft2(out * (Nc / N), norm="ortho").real
