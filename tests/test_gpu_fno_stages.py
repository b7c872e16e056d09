"""Stage-level parity of the FNO kernels.

With BF16-exact inputs and weights, every stage of the forward and backward
passes is read back (FNO_OPT_CAPTURE) and recomputed in FP64 from the GPU's
own BF16 inputs to that stage: the k_x transform, the k_y analysis, the mode
mixing, the k_y synthesis, the layer tail (inverse k_x transform, 1x1
convolution, bias, GELU), the lift and the projection, and in the backward
pass each adjoint and every parameter gradient.  The DFT matrices of the
reference are built here from cos/sin and rounded to BF16 (round to nearest
even), as a BF16 implementation must hold them, so that a stage's reference
differs from the kernel only by the kernel's FP32 accumulation and its
final rounding to BF16.  Bound per element: one BF16 ulp of the reference
plus 1e-5 of the sum of the absolute terms (FP32 accumulation), plus 2^-8 of
that sum for a stage that rounds an intermediate to BF16 inside (the fused
projection's hidden layer, the gradient's GELU' product), plus, where GELU
or GELU' enters, the error of the kernels' erf (Abramowitz and Stegun
7.1.28, absolute error at most 3e-7: GELU(z) within 1.6e-7 |z|, GELU'
within 1.6e-7); FP32 parameter
gradients: 1e-4 of the sum of absolute terms (FP32 sums over up to 3e4
points).  A term dropped in a few modes, a mis-weighted k_x = 0 column or a
wrong sign moves affected elements by about the size of the term, far above
these bounds.  The network-level comparison with the exact FP64 oracle is
in test_gpu_fno.py."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import fno as F

pytestmark = pytest.mark.gpu

SPECIALIZED = F.Config(H=128, W=128, cin=3, cout=2, width=32, modes=16, layers=2, hidden=128)
GENERAL = F.Config(H=32, W=32, cin=3, cout=2, width=8, modes=4, layers=2, hidden=16)
# GELU and GELU' in the kernels use erf from Abramowitz and Stegun 7.1.28
# (absolute error <= 3e-7): a bound of 1.6e-7 |z| on GELU(z), 1.6e-7 on GELU'
ERF_ABS = 1.6e-7


def say(*a):
    print("[case]", *a, flush=True)


def bf16(a):
    """Round to BF16 (through FP32, round to nearest even), as float64."""
    a = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def ulp(x):
    """One BF16 ulp at |x| (8 significant bits)."""
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1e-300)))
    return np.where(ax > 0, 2.0 ** (e - 7), 2.0 ** -133)


def check(name, got, ref, S, inner=0.0, acc=1e-5, abs_tol=0.0):
    tol = ulp(ref) + acc * S + inner * S + abs_tol
    bad = np.abs(got - ref) > tol
    worst = float(np.max(np.abs(got - ref) / ulp(ref)))
    print(f"{name}: max |err| / ulp = {worst:.2f}, {int(bad.sum())} of {bad.size} beyond the bound", flush=True)
    assert not bad.any(), (name, np.argwhere(bad)[:5], got[bad][:5], ref[bad][:5])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def dgelu(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def dft_consts(cfg):
    """The pruned transforms' matrices, from their definitions, in BF16."""
    m, H, W = cfg.modes, cfg.H, cfg.W
    kx = np.arange(m)[:, None]
    x = np.arange(W)[None, :]
    th = 2 * math.pi * kx * x / W
    w = np.where(np.arange(m) == 0, 1.0, 2.0)[:, None] / (H * W)
    Dx = bf16(np.concatenate([np.cos(th), -np.sin(th)]))                  # [2m][W]
    DxG = bf16(np.concatenate([w * np.cos(th), -w * np.sin(th)]))         # [2m][W]
    Ax = bf16(np.concatenate([w * np.cos(th), -w * np.sin(th)]).T)        # [W][2m]
    Ax1 = bf16(np.concatenate([np.cos(th), -np.sin(th)]).T)               # [W][2m]
    ky = np.array([q if q < m else q - 2 * m for q in range(2 * m)])[:, None]
    y = np.arange(H)[None, :]
    ph = 2 * math.pi * ky * y / H                                         # [2m][H]
    DyRe = bf16(np.concatenate([np.cos(ph), -np.sin(ph)]))                # [4m][H]
    DyIm = bf16(np.concatenate([np.sin(ph), np.cos(ph)]))                 # [4m][H]
    Ec, Es = bf16(np.cos(ph).T), bf16(np.sin(ph).T)                       # [H][2m]
    return dict(Dx=Dx, DxG=DxG, Ax=Ax, Ax1=Ax1, DyRe=DyRe, DyIm=DyIm, Ec=Ec, Es=Es)


# ---- the stages, with the sums of absolute terms beside them ------------------------------
def kx_transform(D, h, B, cfg):
    """[B][H][W][C] -> [B][2m][H][C]: sum_x D[k][x] h[b][y][x][c]."""
    h = h.reshape(B, cfg.H, cfg.W, cfg.width)
    return (np.einsum("kx,byxc->bkyc", D, h), np.einsum("kx,byxc->bkyc", np.abs(D), np.abs(h)))


def ky_analysis(T1, c, B, cfg):
    """T1 [B][2m][H][C] -> [m][4m][B][C]: rows q < 2m Re, 2m + q Im of
    sum_y e^{-i k_y y} (T1_re + i T1_im)."""
    m = cfg.modes
    T1 = T1.reshape(B, 2 * m, cfg.H, cfg.width)
    re, im = T1[:, :m], T1[:, m:]
    G = np.einsum("qy,bkyc->kqbc", c["DyRe"], re) + np.einsum("qy,bkyc->kqbc", c["DyIm"], im)
    S = np.einsum("qy,bkyc->kqbc", np.abs(c["DyRe"]), np.abs(re)) + np.einsum("qy,bkyc->kqbc", np.abs(c["DyIm"]),
                                                                                np.abs(im))
    return G, S


def mix(G, R, B, cfg, adjoint=False):
    """G [m][4m][B][C] -> [m][2m][B][2C]: per mode (k_x, k_y row q), R F
    (forward) or R^H g (adjoint), R[q][kx] C x C from the parameters."""
    m, C = cfg.modes, cfg.width
    G = G.reshape(m, 4 * m, B, C)
    gr, gi = G[:, :2 * m], G[:, 2 * m:]
    Rr = np.transpose(R.real, (1, 0, 2, 3))  # [kx][q][c][o]
    Ri = np.transpose(R.imag, (1, 0, 2, 3))
    if not adjoint:
        o_r = np.einsum("kqbc,kqco->kqbo", gr, Rr) - np.einsum("kqbc,kqco->kqbo", gi, Ri)
        o_i = np.einsum("kqbc,kqco->kqbo", gr, Ri) + np.einsum("kqbc,kqco->kqbo", gi, Rr)
        s = np.einsum("kqbc,kqco->kqbo", np.abs(gr), np.abs(Rr)) + np.einsum("kqbc,kqco->kqbo", np.abs(gi), np.abs(Ri))
        s_i = np.einsum("kqbc,kqco->kqbo", np.abs(gr), np.abs(Ri)) + np.einsum("kqbc,kqco->kqbo", np.abs(gi), np.abs(Rr))
    else:
        o_r = np.einsum("kqbo,kqco->kqbc", gr, Rr) + np.einsum("kqbo,kqco->kqbc", gi, Ri)
        o_i = np.einsum("kqbo,kqco->kqbc", gi, Rr) - np.einsum("kqbo,kqco->kqbc", gr, Ri)
        s = np.einsum("kqbo,kqco->kqbc", np.abs(gr), np.abs(Rr)) + np.einsum("kqbo,kqco->kqbc", np.abs(gi), np.abs(Ri))
        s_i = np.einsum("kqbo,kqco->kqbc", np.abs(gi), np.abs(Rr)) + np.einsum("kqbo,kqco->kqbc", np.abs(gr), np.abs(Ri))
    return np.concatenate([o_r, o_i], axis=-1), np.concatenate([s, s_i], axis=-1)


def ky_synthesis(O, c, B, cfg):
    """O [m][2m][B][2C] -> [B][H][2m][C]: sum_q e^{+i k_y y} (O_r + i O_i),
    real part at k_x, imaginary part at m + k_x."""
    m, C = cfg.modes, cfg.width
    O = O.reshape(m, 2 * m, B, 2 * C)
    o_r, o_i = O[..., :C], O[..., C:]
    fr = np.einsum("yq,kqbc->bykc", c["Ec"], o_r) - np.einsum("yq,kqbc->bykc", c["Es"], o_i)
    fi = np.einsum("yq,kqbc->bykc", c["Es"], o_r) + np.einsum("yq,kqbc->bykc", c["Ec"], o_i)
    sr = np.einsum("yq,kqbc->bykc", np.abs(c["Ec"]), np.abs(o_r)) + np.einsum("yq,kqbc->bykc", np.abs(c["Es"]), np.abs(o_i))
    si = np.einsum("yq,kqbc->bykc", np.abs(c["Es"]), np.abs(o_r)) + np.einsum("yq,kqbc->bykc", np.abs(c["Ec"]), np.abs(o_i))
    return np.concatenate([fr, fi], axis=2), np.concatenate([sr, si], axis=2)


def tail(A, T2, hin, Wm, b, B, cfg):
    """[B][H][W][C]: sum_k A[x][k] T2[b][y][k][o] + sum_c hin[..][c] Wm[c][o] + b[o]."""
    H, Wd, C, m = cfg.H, cfg.W, cfg.width, cfg.modes
    T2 = T2.reshape(B, H, 2 * m, C)
    hin = hin.reshape(B, H, Wd, C)
    z = np.einsum("xk,bykc->byxc", A, T2) + np.einsum("byxc,co->byxo", hin, Wm) + b
    S = np.einsum("xk,bykc->byxc", np.abs(A), np.abs(T2)) + np.einsum("byxc,co->byxo", np.abs(hin), np.abs(Wm)) + np.abs(b)
    return z, S


def setup(gpu, cfg, B, seed):
    """A network with BF16-exact parameters and input, one training forward
    (loss against a random target) and backward, with capture on."""
    import torch
    from paper_2304_03306_amd import fno
    net = fno.FNO(width=cfg.width, modes=cfg.modes, layers=cfg.layers, cin=cfg.cin, cout=cfg.cout,
                  hidden=cfg.hidden, H=cfg.H, W=cfg.W, max_batch=B, seed=seed)
    p = F.init_params(cfg, seed)
    rng = np.random.default_rng(seed + 11)
    for k in p:
        if k.startswith("b") or k.endswith("_b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    # weights in BF16 (the kernels' operands); biases stay FP32
    for k in list(p):
        if not (k.startswith("b") or k.endswith("_b")):
            p[k] = bf16(p[k].real) + (1j * bf16(p[k].imag) if np.iscomplexobj(p[k]) else 0.0)
    net.set_params(fno.flatten_params(p, cfg.layers))
    p = fno.unflatten(net.params(), p, cfg.layers)
    net.set_option(fno.FNO_OPT_CAPTURE, 1)
    x = bf16(rng.standard_normal((B, cfg.H, cfg.W, cfg.cin))).astype(np.float32)
    t = rng.standard_normal((B, cfg.H, cfg.W, cfg.cout)).astype(np.float32)
    y = torch.empty((B, cfg.H, cfg.W, cfg.cout), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(x).cuda(), y, train=True)
    net.loss(y, torch.from_numpy(t).cuda())
    net.backward(B)
    torch.cuda.synchronize()
    return net, p, x, y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("cfg", [SPECIALIZED, GENERAL], ids=["specialized", "general"])
def test_forward_stages(gpu, cfg):
    from paper_2304_03306_amd import fno
    B = 2 if cfg is SPECIALIZED else 3
    say("fno forward stages", cfg, B)
    net, p, x, y = setup(gpu, cfg, B, 21)
    c = dft_consts(cfg)
    m, C, H, W, L = cfg.modes, cfg.width, cfg.H, cfg.W, cfg.layers
    P = B * H * W
    nT, nG, nO = B * 2 * m * H * C, m * 4 * m * B * C, m * 2 * m * B * 2 * C
    xb = net.capture(fno.FNO_CAP_XB, 0, P * cfg.cin).reshape(B, H, W, cfg.cin)
    assert np.array_equal(xb, x.astype(np.float64))
    h = [net.capture(fno.FNO_CAP_H, l, P * C) for l in range(L + 1)]
    h0, S = np.einsum("byxk,kc->byxc", xb, p["P_w"]) + p["P_b"], np.einsum("byxk,kc->byxc", np.abs(xb), np.abs(p["P_w"])) + np.abs(p["P_b"])
    check("lift", h[0], h0.ravel(), S.ravel())
    for l in range(L):
        T1 = net.capture(fno.FNO_CAP_T1, l, nT)
        ref, S = kx_transform(c["Dx"], h[l], B, cfg)
        check(f"layer {l} k_x transform", T1, ref.ravel(), S.ravel())
        G = net.capture(fno.FNO_CAP_G, l, nG)
        ref, S = ky_analysis(T1, c, B, cfg)
        check(f"layer {l} k_y analysis", G, ref.ravel(), S.ravel())
        O = net.capture(fno.FNO_CAP_O, l, nO)
        ref, S = mix(G, p[f"R{l}"], B, cfg)
        check(f"layer {l} mode mixing", O, ref.ravel(), S.ravel())
        T2 = net.capture(fno.FNO_CAP_T2, l, nT)
        ref, S = ky_synthesis(O, c, B, cfg)
        check(f"layer {l} k_y synthesis", T2, ref.ravel(), S.ravel())
        z, S = tail(c["Ax"], T2, h[l], p[f"W{l}"], p[f"b{l}"], B, cfg)
        if l < L - 1:
            zg = net.capture(fno.FNO_CAP_Z, l, P * C)
            check(f"layer {l} pre-activation", zg, z.ravel(), S.ravel())
            # GELU of the FP32 pre-activation, rounded once
            check(f"layer {l} GELU", h[l + 1], gelu(z).ravel(), (np.abs(dgelu(z)) * S).ravel(),
                  abs_tol=ERF_ABS * np.abs(z).ravel())
        else:
            check(f"layer {l} output", h[l + 1], z.ravel(), S.ravel())
    # projection: the hidden layer GELU(h_L Q1 + b1) is rounded to BF16 inside
    hL = h[L].reshape(P, C)
    u = hL @ p["Q1_w"] + p["Q1_b"]
    a = gelu(u)
    ref = (a @ p["Q2_w"] + p["Q2_b"]).ravel()
    S = (np.abs(a) @ np.abs(p["Q2_w"]) + np.abs(p["Q2_b"])).ravel()
    check("projection", y.ravel(), ref, S, inner=2.0 ** -8,
          abs_tol=ERF_ABS * (np.abs(u) @ np.abs(p["Q2_w"])).ravel())


@pytest.mark.parametrize("cfg", [SPECIALIZED, GENERAL], ids=["specialized", "general"])
def test_backward_stages(gpu, cfg):
    from paper_2304_03306_amd import fno
    B = 2 if cfg is SPECIALIZED else 3
    say("fno backward stages", cfg, B)
    net, p, x, y = setup(gpu, cfg, B, 23)
    c = dft_consts(cfg)
    m, C, H, W, L = cfg.modes, cfg.width, cfg.H, cfg.W, cfg.layers
    P = B * H * W
    nT, nG, nO = B * 2 * m * H * C, m * 4 * m * B * C, m * 2 * m * B * 2 * C
    g = fno.unflatten(net.grads(), p, L)
    h = [net.capture(fno.FNO_CAP_H, l, P * C).reshape(P, C) for l in range(L + 1)]
    xb = net.capture(fno.FNO_CAP_XB, 0, P * cfg.cin).reshape(P, cfg.cin)
    dy = net.capture(fno.FNO_CAP_DY, 0, P * cfg.cout).reshape(P, cfg.cout)
    # projection backward: dh_L = ((dy Q2^T) GELU'(u)) Q1^T, du rounded to BF16 inside
    u = h[L] @ p["Q1_w"] + p["Q1_b"]
    du = (dy @ p["Q2_w"].T) * dgelu(u)
    # scale of du's rounding: GELU' may be taken at the BF16-stored
    # pre-activation (|GELU''| <= 0.8), and du is rounded to BF16
    Sdu = (np.abs(dy) @ np.abs(p["Q2_w"]).T) * (np.abs(dgelu(u)) + 0.4 * np.abs(u))
    dhL = net.capture(fno.FNO_CAP_DHL, 0, P * C)
    check("projection backward dl/dh_L", dhL, (du @ p["Q1_w"].T).ravel(), (Sdu @ np.abs(p["Q1_w"]).T).ravel(),
          inner=2.0 ** -8)
    a = gelu(u)
    tol = lambda S: 1e-4 * S + 1e-6 * np.abs(S).max()
    for name, ref, S in (("Q2_w", a.T @ dy, np.abs(a).T @ np.abs(dy)), ("Q2_b", dy.sum(0), np.abs(dy).sum(0))):
        err = np.abs(g[name] - ref)
        print(f"grad {name}: max err / sum|terms| = {float(np.max(err / (S + 1e-300))):.2e}", flush=True)
        assert (err <= 2.0 ** -8 * S + tol(S)).all(), name  # a is rounded to BF16 as an operand
    for name, ref, S in (("Q1_w", h[L].T @ du, np.abs(h[L]).T @ Sdu), ("Q1_b", du.sum(0), Sdu.sum(0))):
        err = np.abs(g[name] - ref)
        print(f"grad {name}: max err / sum|terms| = {float(np.max(err / (S + 1e-300))):.2e}", flush=True)
        assert (err <= 2.0 ** -8 * S + tol(S)).all(), name  # du is rounded to BF16 as an operand
    for l in reversed(range(L)):
        dz = net.capture(fno.FNO_CAP_DZ, l, P * C)
        if l == L - 1:
            assert np.array_equal(dz, dhL)
        else:
            assert np.array_equal(dz, net.capture(fno.FNO_CAP_DH, l + 1, P * C))
        dzm = dz.reshape(P, C)
        for name, ref, S in ((f"W{l}", h[l].T @ dzm, np.abs(h[l]).T @ np.abs(dzm)),
                             (f"b{l}", dzm.sum(0), np.abs(dzm).sum(0))):
            err = np.abs(g[name] - ref)
            print(f"grad {name}: max err / sum|terms| = {float(np.max(err / (S + 1e-300))):.2e}", flush=True)
            assert (err <= tol(S)).all(), name
        BT1 = net.capture(fno.FNO_CAP_BT1, l, nT)
        ref, S = kx_transform(c["DxG"], dz, B, cfg)
        check(f"layer {l} adjoint k_x transform", BT1, ref.ravel(), S.ravel())
        gG = net.capture(fno.FNO_CAP_GG, l, nG)
        ref, S = ky_analysis(BT1, c, B, cfg)
        check(f"layer {l} adjoint k_y analysis", gG, ref.ravel(), S.ravel())
        # dR per mode from the forward modes F (G) and gG
        Gf = net.capture(fno.FNO_CAP_G, l, nG).reshape(m, 4 * m, B, C)
        gg = gG.reshape(m, 4 * m, B, C)
        fr, fi, gr, gi = Gf[:, :2 * m], Gf[:, 2 * m:], gg[:, :2 * m], gg[:, 2 * m:]
        dRr = np.einsum("kqbc,kqbo->qkco", fr, gr) + np.einsum("kqbc,kqbo->qkco", fi, gi)
        dRi = np.einsum("kqbc,kqbo->qkco", fr, gi) - np.einsum("kqbc,kqbo->qkco", fi, gr)
        SR = np.einsum("kqbc,kqbo->qkco", np.abs(fr), np.abs(gr)) + np.einsum("kqbc,kqbo->qkco", np.abs(fi), np.abs(gi))
        SI = np.einsum("kqbc,kqbo->qkco", np.abs(fr), np.abs(gi)) + np.einsum("kqbc,kqbo->qkco", np.abs(fi), np.abs(gr))
        for name, got, ref, S in ((f"R{l} real", g[f"R{l}"].real, dRr, SR), (f"R{l} imag", g[f"R{l}"].imag, dRi, SI)):
            err = np.abs(got - ref)
            print(f"grad {name}: max err / sum|terms| = {float(np.max(err / (S + 1e-300))):.2e}", flush=True)
            assert (err <= tol(S)).all(), name
        gF = net.capture(fno.FNO_CAP_GF, l, nO)
        ref, S = mix(gG, p[f"R{l}"], B, cfg, adjoint=True)
        check(f"layer {l} adjoint mode mixing", gF, ref.ravel(), S.ravel())
        BT2 = net.capture(fno.FNO_CAP_BT2, l, nT)
        ref, S = ky_synthesis(gF, c, B, cfg)
        check(f"layer {l} adjoint k_y synthesis", BT2, ref.ravel(), S.ravel())
        dh, S = tail(c["Ax1"], BT2, dzm, p[f"W{l}"].T, 0.0, B, cfg)
        DH = net.capture(fno.FNO_CAP_DH, l, P * C)
        if l > 0:
            zp = net.capture(fno.FNO_CAP_Z, l - 1, P * C).reshape(dh.shape)
            check(f"layer {l} gradient handed down (x GELU')", DH, (dh * dgelu(zp)).ravel(),
                  (S * np.abs(dgelu(zp))).ravel(), inner=2.0 ** -8, abs_tol=ERF_ABS * S.ravel())
        else:
            check(f"layer {l} gradient handed down", DH, dh.ravel(), S.ravel())
    dh0 = net.capture(fno.FNO_CAP_DH, 0, P * C).reshape(P, C)
    for name, ref, S in (("P_w", xb.T @ dh0, np.abs(xb).T @ np.abs(dh0)), ("P_b", dh0.sum(0), np.abs(dh0).sum(0))):
        err = np.abs(g[name] - ref)
        print(f"grad {name}: max err / sum|terms| = {float(np.max(err / (S + 1e-300))):.2e}", flush=True)
        assert (err <= tol(S)).all(), name
