"""Training and evaluation loop of the learned short-window path.

Every step runs in libqld's kernels (pair generation, normalisation, target,
forward, backward, Adam, judges); this module only sequences the calls and
draws the seeded scene parameters and initial weights on the host (they are
inputs).  Plain QLD is the fallback and the judge:

* training pairs: short window (M_S cycles) I/Q in, bias-reduced long-window
  (M_L cycles) amplitude out, of the same generated stack;
* gate target: the tile's excess error NRMSE(learned) - NRMSE(plain at M_L),
  both against the per-cycle lock-in amplitude of the noise-free rates;
* serving rule: learned output when the predicted excess is at most
  ``gate_threshold``, plain QLD at M_L otherwise.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import paper_1511_03390_amd as qld
import scenes

LAYERS = ((2, 32), (32, 32), (32, 32), (32, 1))


def he_init(seed):
    """He-normal weights, zero biases and gate, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in LAYERS:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=9 * ci * co))
        parts.append(np.zeros(co))
    parts.append(np.zeros(33))
    return np.concatenate(parts).astype(np.float32)


class Batch:
    """Device tensors of one batch of generated tiles."""

    def __init__(self, params, M_S, M_L, tile0, seed, bits=12):
        self.mask = torch.from_numpy(params["mask"]).cuda()
        self.rates = params["rates"]
        self.M_S, self.M_L = M_S, M_L
        (self.I_S, self.Q_S, self.I_L, self.Q_L, self.sum_S, self.sum_L, self.psum_S,
         self.psum_L) = qld.gen_pairs(self.mask, self.rates, M_S, M_L, tile0, seed, bits)
        self.x, self.scale = qld.denoise_prepare(self.I_S, self.Q_S, self.psum_S, self.sum_S, M_S)
        self.t = qld.denoise_target(self.I_L, self.Q_L, self.psum_L, M_L, self.scale)
        self.clean = qld.clean_amplitude(self.mask, self.rates)
        B, H, W = self.I_S.shape
        self.B, self.H, self.W = B, H, W
        self.ampL = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
        qld.amplitude(self.I_L, self.Q_L, self.ampL)
        self.ampS = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
        qld.amplitude(self.I_S, self.Q_S, self.ampS)
        self.invL = torch.full((B,), 1.0 / M_L, dtype=torch.float32, device="cuda")
        self.invS = torch.full((B,), 1.0 / M_S, dtype=torch.float32, device="cuda")

    def record_stream(self, stream):
        """Mark every device tensor as used on ``stream`` (made on another
        stream), so its memory is not reused before that stream's work on it."""
        for v in vars(self).values():
            if isinstance(v, torch.Tensor) and v.is_cuda:
                v.record_stream(stream)


TILES_CONFIG4 = dict(background=2000.0, ballistic=5e-4, smin=16, smax=256, max_rects=5)


def tile_batch(step, batch, H, W, M_S, M_L, seed, tiles=None):
    """Generated batch number ``step``: scene parameters from the tile recipe
    ``tiles`` (keyword arguments of scenes.tile_params; default: 1-5 rectangles
    of sides 16-256 at ballistic fraction 5e-4 of a 2000-count background)."""
    p = scenes.tile_params(scenes.seed_for(4, step), batch, H=H, W=W, **(tiles or TILES_CONFIG4))
    return Batch(p, M_S, M_L, tile0=step * batch, seed=seed)


def train(steps=200, batch=8, H=512, W=512, M_S=8, M_L=512, lr=2e-3, seed=1511033904, gate_weight=0.1,
          log=None, first_step=0, tiles=None):
    """Train on generated batches.  Batch s + 1 is generated on a second
    stream while step s trains (the generator is bound by its VALU work, the
    training by memory and the matrix cores); an event orders each step after
    its batch.  The steps and their results are those of generating and
    training one after the other."""
    d = qld.Denoiser(H, W, batch)
    d.set_params(he_init(seed))
    y = torch.empty((batch, H, W), dtype=torch.float32, device="cuda")
    loss = torch.zeros(2, dtype=torch.float32, device="cuda")
    hist = []
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()

    def generate(s):
        with torch.cuda.stream(side):
            b = tile_batch(first_step + s, batch, H, W, M_S, M_L, seed, tiles)
            done = torch.cuda.Event()
            done.record(side)
        return b, done

    t0 = time.perf_counter()
    nxt = generate(0) if steps > 0 else None
    for s in range(steps):
        b, done = nxt
        main.wait_event(done)
        b.record_stream(main)
        if s + 1 < steps:
            nxt = generate(s + 1)
        d.forward(b.x, y)
        nl = qld.judge_nrmse(y, b.clean, b.scale)
        npl = qld.judge_nrmse(b.ampL, b.clean, b.invL)
        d.backward(b.t, nl, npl, gate_weight, loss)
        d.adam(lr)
        if s % max(1, steps // 10) == 0 or s == steps - 1:
            lv = loss.cpu().numpy()
            hist.append((s, float(lv[0]), float(lv[1])))
            if log:
                log("step %d loss %.5f gate %.5f" % (s, lv[0], lv[1]))
    torch.cuda.synchronize()
    return d, hist, time.perf_counter() - t0


def evaluate(d, n_batches=2, batch=8, H=512, W=512, M_S=8, M_L=512, seed=1511033904, first_step=10 ** 6,
             gate_threshold=0.05, tiles=None):
    """NRMSE against the noise-free per-cycle amplitude on held-out tiles."""
    y = torch.empty((batch, H, W), dtype=torch.float32, device="cuda")
    gate = torch.empty(batch, dtype=torch.float32, device="cuda")
    acc = {k: [] for k in ("learned", "plain_S", "plain_L", "plain_L_bias_reduced", "served", "gate",
                           "learned_vs_noisy_L", "cnr_learned", "cnr_plain_S", "cnr_plain_L")}

    def tile_cnr(img, m):
        """(mean over the mask - mean outside) / std outside, per tile: the
        contrast a detector sees (0 for an image that ignores the scene)."""
        m = m.bool()
        out = []
        for i in range(img.shape[0]):
            a, bg = img[i][m[i]], img[i][~m[i]]
            out.append(float(((a.mean() - bg.mean()) / bg.std()).item()) if a.numel() and bg.numel() > 1 else 0.0)
        return np.array(out)

    for k in range(n_batches):
        b = tile_batch(first_step + k, batch, H, W, M_S, M_L, seed, tiles)
        d.forward(b.x, y, gate)
        acc["learned"].append(qld.judge_nrmse(y, b.clean, b.scale).cpu().numpy())
        acc["plain_S"].append(qld.judge_nrmse(b.ampS, b.clean, b.invS).cpu().numpy())
        acc["plain_L"].append(qld.judge_nrmse(b.ampL, b.clean, b.invL).cpu().numpy())
        acc["plain_L_bias_reduced"].append(qld.judge_nrmse(b.t, b.clean, b.scale).cpu().numpy())
        acc["cnr_learned"].append(tile_cnr(y, b.mask))
        acc["cnr_plain_S"].append(tile_cnr(b.ampS, b.mask))
        acc["cnr_plain_L"].append(tile_cnr(b.ampL, b.mask))
        ampL_pc = b.ampL * b.invL[:, None, None]
        acc["learned_vs_noisy_L"].append(qld.judge_nrmse(y, ampL_pc, b.scale).cpu().numpy())
        g = gate.cpu().numpy()
        acc["gate"].append(g)
        acc["served"].append(np.where(g > gate_threshold, acc["plain_L"][-1], acc["learned"][-1]))
    per_tile = {k: np.concatenate(v) for k, v in acc.items()}
    out = {k: float(np.mean(v)) for k, v in per_tile.items()}
    out["fallback_rate"] = float(np.mean(per_tile["gate"] > gate_threshold))
    out["tiles"] = n_batches * batch
    out["per_tile"] = per_tile
    return out


def flops_per_pixel_step():
    """Multiply-adds x 2 of one training step per pixel: forward (18x32 + 2 x 288x32
    + 288 MACs) and backward (input gradients of layers 2-4 and weight
    gradients of all four layers, each the size of the forward layer)."""
    fwd = 2 * (18 * 32 + 2 * 288 * 32 + 288)
    bwd_data = 2 * (2 * 288 * 32 + 288)
    bwd_weight = fwd
    return fwd + bwd_data + bwd_weight
