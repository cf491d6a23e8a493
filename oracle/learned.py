"""Oracle of the learned short-window path: training pairs, clean target,
denoiser forward/backward, Adam, gate.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Double precision,
numpy; a matrix product serves as a step of the convolution.

The denoiser is not in the paper: it maps the quadrature sums of a short
window (M_S cycles) to the lock-in amplitude of a long window (M_L cycles)
of the same scene, with plain QLD as its fallback and judge.

Network (NHWC, 3x3 kernels, zero "same" padding, correlation):
    x  = (I_S, Q_S) / sqrt(P_S / 2) per pixel, P_S = the pixel's sample sum over the short window
    s  = sigma / sqrt(M_S),  sigma^2 = 2 * mean sample level of the tile's short window
    a1 = relu(conv(x,  W1) + b1)        2 -> 32
    a2 = relu(conv(a1, W2) + b2)       32 -> 32
    a3 = relu(conv(a2, W3) + b3)       32 -> 32
    y  = conv(a3, W4) + b4             32 -> 1     (per-cycle amplitude / s, s = sigma / sqrt(M_S))
    gate = mean_pixels(a3) . Wg + bg                (predicted excess NRMSE of the tile)
With ``emulate=True`` the values are rounded to bfloat16 (round to nearest
even) where the GPU stores them in bfloat16: the input, the weights, the
hidden activations, and the hidden-layer gradients dz used as operands.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

import oracle as _o

# ---------------------------------------------------------------------------
# Training pairs
# ---------------------------------------------------------------------------


def philox4x32_10(ctr, key):
    lib = _o._load()
    C = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    K = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    O = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32(C, K, 10, O)
    return [int(v) for v in O]


def poisson_table(lam):
    """(lo, thr uint32[hi-lo]) of the inversion table for rate lam."""
    lib = _o._load()
    lo, hi = ctypes.c_int32(), ctypes.c_int32()
    lib.oracle_poisson_bounds(float(lam), ctypes.byref(lo), ctypes.byref(hi))
    thr = np.zeros(hi.value - lo.value + 1, dtype=np.uint32)
    n = lib.oracle_poisson_table(float(lam), thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, thr[:n]


def poisson_invert(lo, thr, u):
    """X(u) = lo + #{thr <= u} (vectorised over u)."""
    return lo + np.searchsorted(thr, np.asarray(u, dtype=np.uint64), side="right")


def gen_frames(mask, rates, n_cycles, tile0, seed, bits=12):
    """Frames [n][4*n_cycles][H][W] uint16 of the tiles (mask [n][H][W], rates [n][2][4])."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    n, H, W = mask.shape
    out = np.zeros((n, 4 * n_cycles, H, W), dtype=np.uint16)
    rc = _o._load().oracle_gen_frames(mask.ctypes.data, rates.ctypes.data, n, H, W, n_cycles,
                                      int(tile0) & 0xFFFFFFFF, int(seed) & 0xFFFFFFFF,
                                      (int(seed) >> 32) & 0xFFFFFFFF, bits, out.ctypes.data)
    if rc:
        raise RuntimeError("oracle_gen_frames failed")
    return out


def gen_pixel_series(pix, mk, rates_tile, n_cycles, tile, seed, bits=12):
    """Series [k][4*n_cycles] uint16 of selected pixels (index y*W + x, mask state mk) of one tile."""
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    mk = np.ascontiguousarray(mk, dtype=np.uint8)
    r = np.ascontiguousarray(rates_tile, dtype=np.float64).reshape(8)
    out = np.zeros((len(pix), 4 * n_cycles), dtype=np.uint16)
    rc = _o._load().oracle_gen_pixels(pix.ctypes.data, mk.ctypes.data, len(pix), r.ctypes.data, n_cycles,
                                      int(tile) & 0xFFFFFFFF, int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF,
                                      bits, out.ctypes.data)
    if rc:
        raise RuntimeError("oracle_gen_pixels failed")
    return out


def gen_pairs(mask, rates, M_S, M_L, tile0, seed, bits=12):
    """Quadrature sums of the short (first M_S cycles) and long (first M_L
    cycles) windows of the generated stack, by the lock-in oracle, plus the
    sample sums of both windows.  Returns dict of int64 arrays [n][H][W] / [n]."""
    fr = gen_frames(mask, rates, M_L, tile0, seed, bits)
    n = fr.shape[0]
    out = {k: [] for k in ("I_S", "Q_S", "I_L", "Q_L", "sum_S", "sum_L", "psum_S", "psum_L")}
    for i in range(n):
        I, Q = _o.qld(fr[i, :4 * M_S])
        out["I_S"].append(I)
        out["Q_S"].append(Q)
        I, Q = _o.qld(fr[i])
        out["I_L"].append(I)
        out["Q_L"].append(Q)
        out["psum_S"].append(fr[i, :4 * M_S].astype(np.int64).sum(axis=0))
        out["psum_L"].append(fr[i].astype(np.int64).sum(axis=0))
        out["sum_S"].append(int(out["psum_S"][-1].sum()))
        out["sum_L"].append(int(out["psum_L"][-1].sum()))
    return {k: np.array(v) for k, v in out.items()}


def a_star(mask, rates):
    """Per-cycle lock-in amplitude of the noise-free expected stack: the
    quadrature sums of one cycle of rates (reference tables exact), then R."""
    c, s = _o.reference_tables()
    lam = np.where(np.asarray(mask)[:, None, :, :] > 0, np.asarray(rates)[:, 1, :, None, None],
                   np.asarray(rates)[:, 0, :, None, None])            # [n][4][H][W]
    I = sum(lam[:, j] * c[j] for j in range(4))
    Q = sum(lam[:, j] * s[j] for j in range(4))
    return np.sqrt(I * I + Q * Q)


def normalise(I_S, Q_S, psum_S, sum_S, M_S, H, W):
    """Network input [n][H][W][2] and output scale s (per tile) from the short window.

    Input: each pixel's (I, Q) over the noise standard deviation of its own
    quadrature sums.  For Poisson light of rate lam at a pixel, every cycle
    adds S0 - S2 of variance 2 lam to I (and S1 - S3 to Q): Var(I) = Var(Q) =
    2 M_S lam; the pixel's sample sum P over the window's 4 M_S frames
    estimates 4 M_S lam, so the divisor is sqrt(P / 2) (x = 0 where P = 0).
    Output scale: sigma / sqrt(M_S), sigma^2 = 2 b, b = the tile's mean sample
    level (its sample sum over H * W * 4 * M_S samples)."""
    ps = np.asarray(psum_S, dtype=np.float64)
    den = np.sqrt(ps / 2.0)
    ok = den > 0
    safe = np.where(ok, den, 1.0)
    x = np.stack([np.where(ok, np.asarray(I_S, dtype=np.float64) / safe, 0.0),
                  np.where(ok, np.asarray(Q_S, dtype=np.float64) / safe, 0.0)], axis=-1)
    b = np.asarray(sum_S, dtype=np.float64) / (H * W * 4 * M_S)       # mean sample level of the tile
    sigma = np.sqrt(2.0 * b)
    return x, sigma / math.sqrt(M_S)


def target(I_L, Q_L, psum_L, M_L, scale):
    """Bias-reduced long-window amplitude per cycle, in units of ``scale``:
    sqrt(max(I^2 + Q^2 - P_L, 0)) / M_L per pixel, P_L = the pixel's sample sum
    over the long window (for Poisson light of rate lam, E[I^2 + Q^2] without
    signal is 4 M_L lam, which P_L estimates)."""
    r2 = np.asarray(I_L, dtype=np.float64) ** 2 + np.asarray(Q_L, dtype=np.float64) ** 2
    t = np.sqrt(np.maximum(r2 - np.asarray(psum_L, dtype=np.float64), 0.0)) / M_L
    return t / np.asarray(scale)[:, None, None]


# ---------------------------------------------------------------------------
# Denoiser
# ---------------------------------------------------------------------------

LAYERS = ((2, 32), (32, 32), (32, 32), (32, 1))
N_PARAMS = sum(9 * ci * co + co for ci, co in LAYERS)   # 19,393


def bf16(x):
    """Round to bfloat16 (nearest even), via float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed):
    """He-normal weights, zero biases, gate zero; weights as [3][3][Cin][Cout]."""
    rng = np.random.default_rng(seed)
    p = {}
    for l, (ci, co) in enumerate(LAYERS, start=1):
        p["W%d" % l] = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=(3, 3, ci, co))
        p["b%d" % l] = np.zeros(co)
    p["Wg"] = np.zeros(32)
    p["bg"] = np.zeros(1)
    return p


def conv(x, w, b=None):
    """3x3 correlation with zero padding: out[p] = sum_tap x[p + tap - 1] @ w[tap]."""
    B, H, W, _ = x.shape
    xp = np.zeros((B, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.zeros((B, H, W, w.shape[3]))
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ w[dy, dx]
    return out if b is None else out + b


def conv_back_data(dz, w):
    """Gradient of conv with respect to its input."""
    B, H, W, _ = dz.shape
    dxp = np.zeros((B, H + 2, W + 2, w.shape[2]))
    for dy in range(3):
        for dx in range(3):
            dxp[:, dy:dy + H, dx:dx + W, :] += dz @ w[dy, dx].T
    return dxp[:, 1:H + 1, 1:W + 1]


def conv_back_weight(x, dz):
    """Gradient of conv with respect to its weights [3][3][Cin][Cout]."""
    B, H, W, ci = x.shape
    xp = np.zeros((B, H + 2, W + 2, ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    dw = np.zeros((3, 3, ci, dz.shape[3]))
    for dy in range(3):
        for dx in range(3):
            dw[dy, dx] = np.einsum("bhwi,bhwo->io", xp[:, dy:dy + H, dx:dx + W, :], dz)
    return dw


def forward(p, x, emulate=True):
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    act = {"x0": r(x)}
    h = act["x0"]
    for l in (1, 2, 3):
        z = conv(h, r(p["W%d" % l]), p["b%d" % l])
        h = r(np.maximum(z, 0.0))
        act["a%d" % l] = h
    y = conv(h, r(p["W4"]), p["b4"])[..., 0]
    act["y"] = y
    g = act["a3"].mean(axis=(1, 2))                      # [B][32]
    act["pool"] = g
    act["gate"] = g @ p["Wg"] + p["bg"][0]
    return act


def loss_and_grads(p, x, t, e=None, gate_weight=1.0, emulate=True):
    """Mean squared error of y against t, with the explicit backward pass for
    the trunk (W1..b4); and the gate's own loss, gate_weight * mean (gate - e)^2,
    whose gradient reaches only Wg, bg (the trunk's features are constants to
    it).  Returns (loss, gate_loss, grads, activations)."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    act = forward(p, x, emulate)
    B, H, W = t.shape
    n = B * H * W
    y = act["y"]
    loss = float(np.mean((y - t) ** 2))
    g = {}
    dy = (2.0 / n) * (y - t)
    dz = dy[..., None]
    h_in = {1: act["x0"], 2: act["a1"], 3: act["a2"], 4: act["a3"]}
    for l in (4, 3, 2, 1):
        w = r(p["W%d" % l])
        g["W%d" % l] = conv_back_weight(h_in[l], dz)
        g["b%d" % l] = dz.sum(axis=(0, 1, 2))
        if l > 1:
            da = conv_back_data(dz, w)
            dz = r(da * (h_in[l] > 0))
    gate_loss = 0.0
    if e is not None:
        de = gate_weight * (2.0 / B) * (act["gate"] - np.asarray(e))
        gate_loss = gate_weight * float(np.mean((act["gate"] - np.asarray(e)) ** 2))
        g["Wg"] = act["pool"].T @ de
        g["bg"] = np.array([de.sum()])
    else:
        g["Wg"] = np.zeros(32)
        g["bg"] = np.zeros(1)
    return loss, gate_loss, g, act


def adam(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015), bias-corrected, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
