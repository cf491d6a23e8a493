"""Seeded synthetic camera scenes: the inputs shared by the HIP path and the oracle.

This module only *renders inputs* (frame stacks, scene parameters, Poisson rates).
It holds none of the lock-in arithmetic: no I/Q sums, no amplitude, no DFT.
Both the product package and the CPU oracle are fed from here; neither imports
the other.

The paper's own recordings and its simulation parameters (frame size, source
size, sampling interval, seeds) are not available, so these generators stand
in for them.  They follow the paper's simulation recipe (Methods, "Numerical
simulations": modulated sources on a diffuse, noisy background, one intensity
series per pixel) and its experimental setting (16-bit camera frames, sources
modulated at the lock-in frequency, four samples per modulation period).

Layout of every stack: ``[T][H][W]`` row-major, time-major (one frame after the
other), dtype uint8 or uint16 (12-bit values in a uint16 container where stated).
Frame ``t`` has lock-in phase ``(phase0 + t) mod 4``; all generators here use
``phase0 = 0``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 1511033900


def seed_for(config: int, sub: int = 0) -> int:
    """Seed of configuration ``config`` (1..5), sub-stream ``sub``."""
    return SEED_BASE + config + 1000 * sub


@dataclasses.dataclass
class Stack:
    frames: object            # np.ndarray or torch.Tensor, [T][H][W]
    bits: int                 # significant bits per sample (8, 12 or 16)
    meta: dict

    @property
    def T(self):
        return int(self.frames.shape[0])


def _disk_mask(H, W, cy, cx, r):
    yy, xx = np.mgrid[0:H, 0:W]
    return (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r


def square_wave(t, phi):
    """+1 where cos(pi t / 2 + phi) >= 0, else -1 (four samples per period)."""
    return np.where(np.cos(np.pi * np.asarray(t, dtype=np.float64) / 2.0 + phi) >= 0.0, 1.0, -1.0)


# ---------------------------------------------------------------------------
# Small batch scene: 64x64 uint8, M = 16 cycles.
# ---------------------------------------------------------------------------
def disk_scene_u8(seed=None, H=64, W=64, M=16, background=100.0, sigma=8.0,
                  radius=12, amplitude=4.0, center=None):
    """Background + Gaussian noise, one square-wave modulated disk, uint8 frames.

    The disk adds +amplitude where cos(pi t/2 + phi) >= 0 and -amplitude
    elsewhere; phi ~ U[0, 2 pi).  Values are rounded to nearest (ties to even)
    and clipped to [0, 255].
    """
    if seed is None:
        seed = seed_for(1)
    rng = np.random.default_rng(seed)
    T = 4 * M
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    noise = rng.normal(0.0, sigma, size=(T, H, W))
    cy, cx = center if center is not None else (H // 2, W // 2)
    mask = _disk_mask(H, W, cy, cx, radius)
    sq = square_wave(np.arange(T), phi) * amplitude
    x = background + noise + mask[None, :, :] * sq[:, None, None]
    frames = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    return Stack(frames, 8, dict(phi=phi, mask=mask, M=M, amplitude=amplitude,
                                 background=background, sigma=sigma, seed=seed))


# ---------------------------------------------------------------------------
# Batch scene under strong diffuse light: uint16 with 12-bit values.
# ---------------------------------------------------------------------------
def rect_masks(rng, H, W, n, smin, smax):
    """Union of ``n`` axis-aligned rectangles with sides U{smin..smax}, each fully inside."""
    mask = np.zeros((H, W), dtype=bool)
    rects = []
    for _ in range(n):
        h = int(rng.integers(smin, min(smax, H) + 1))
        w = int(rng.integers(smin, min(smax, W) + 1))
        y0 = int(rng.integers(0, H - h + 1))
        x0 = int(rng.integers(0, W - w + 1))
        mask[y0:y0 + h, x0:x0 + w] = True
        rects.append((y0, x0, h, w))
    return mask, rects


def diffuse_scene_params(seed=None, H=1024, W=1024, T=1024, background=2000.0,
                         ballistic=1e-3, drift=50.0, n_rects=5, smin=32, smax=256):
    """Parameters of the diffuse scene: mask, phase, per-frame offset and rate terms.

    Rate of pixel p in frame t:
        lam = background + d(t) + mask(p) * ballistic * background * (1 + cos(pi t / 2 + phi)),
        d(t) = -drift + 2 * drift * t / (T - 1)   (linear ambient drift).
    """
    if seed is None:
        seed = seed_for(2)
    rng = np.random.default_rng(seed)
    smax_eff = max(smin, min(smax, H, W))
    mask, rects = rect_masks(rng, H, W, n_rects, min(smin, smax_eff), smax_eff)
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    t = np.arange(T, dtype=np.float64)
    d = -drift + 2.0 * drift * t / max(T - 1, 1)
    mod = ballistic * background * (1.0 + np.cos(np.pi * t / 2.0 + phi))
    return dict(seed=seed, mask=mask, rects=rects, phi=phi, offset=background + d,
                modulation=mod, H=H, W=W, T=T, bits=12, background=background,
                ballistic=ballistic)


def diffuse_scene_u16(seed=None, H=1024, W=1024, T=1024, device="cpu", chunk=64, frame_stride=None, **kw):
    """Poisson frames of the diffuse scene as a torch int16 tensor holding uint16 bits.

    Drawn with ``torch.poisson`` from a seeded ``torch.Generator`` on ``device``
    (the same seed on CPU and GPU gives different, equally valid stacks), then
    clipped to the 12-bit range.  Generated ``chunk`` frames at a time to bound
    memory.  ``frame_stride`` (elements, >= H*W) lays the frames out with gaps
    between them (a [T][H][W] view of a larger buffer); the values do not
    depend on it.  Returns a :class:`Stack` whose ``frames`` is a torch tensor.
    """
    import torch

    p = diffuse_scene_params(seed, H, W, T, **kw)
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(p["seed"]))
    mask = torch.from_numpy(p["mask"].astype(np.float32)).to(dev)
    fs = H * W if frame_stride is None else int(frame_stride)
    if fs < H * W:
        raise ValueError("frame_stride %d < H*W = %d" % (fs, H * W))
    if fs == H * W:
        out = torch.empty((T, H, W), dtype=torch.int16, device=dev)
    else:
        out = torch.zeros(T * fs, dtype=torch.int16, device=dev).as_strided((T, H, W), (fs, W, 1))
    maxv = float((1 << p["bits"]) - 1)
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        off = torch.tensor(p["offset"][t0:t1], dtype=torch.float32, device=dev)
        mod = torch.tensor(p["modulation"][t0:t1], dtype=torch.float32, device=dev)
        lam = off[:, None, None] + mask[None] * mod[:, None, None]
        x = torch.poisson(lam, generator=g).clamp_(0.0, maxv)
        out[t0:t1] = x.to(torch.int32).to(torch.int16)
    return Stack(out, p["bits"], p)


def random_stack(rng, T, H, W, dtype, bits=None, lo=0, hi=None, pitch=None):
    """Uniform random integer frames; ``pitch`` > W gives padded rows (padding = 0xA5 bytes).

    Returns (buffer, view): ``buffer`` is the full [T][H][pitch] array,
    ``view`` the [T][H][W] window of it.
    """
    dt = np.dtype(dtype)
    if bits is None:
        bits = dt.itemsize * 8
    if hi is None:
        hi = (1 << bits) - 1
    pitch = W if pitch is None else pitch
    buf = np.full((T, H, pitch), 0xA5A5 & ((1 << (8 * dt.itemsize)) - 1), dtype=dt)
    buf[:, :, :W] = rng.integers(lo, hi + 1, size=(T, H, W), dtype=np.int64).astype(dt)
    return buf, buf[:, :, :W]


# ---------------------------------------------------------------------------
# Streaming cameras: the small-scene content on large uint16 frames, plus a
# modulated disk that translates by one pixel per cycle (wrapping in x).
# ---------------------------------------------------------------------------
class CameraStream:
    """A seeded camera that produces one cycle (four frames) at a time.

    Content: background 100 + N(0, 8^2) noise, ``n_static`` square-wave disks
    (radius 12, amplitude 4, one random phase each) at fixed random places, and
    one disk of the same kind whose centre moves +1 px in x every cycle with
    wrap-around.  Noise comes from a bank of ``bank`` pre-drawn frames reused
    cyclically (frame t uses bank entry t mod bank), so frames can be produced
    at camera rate; every other term is exact per frame.  Rounded to nearest
    and clipped to [0, 2^bits - 1].
    """

    def __init__(self, H, W, seed, bits=16, n_static=3, radius=12, amplitude=4.0,
                 background=100.0, sigma=8.0, bank=16):
        self.H, self.W, self.bits, self.seed = H, W, bits, seed
        rng = np.random.default_rng(seed)
        self.radius, self.amplitude = radius, amplitude
        self.noise = np.rint(background + rng.normal(0.0, sigma, size=(bank, H, W))).astype(np.int32)
        self.static = []

        def centre(n):
            # Keep the disk inside when the frame is large enough; otherwise anywhere.
            return int(rng.integers(radius, n - radius)) if n > 2 * radius else int(rng.integers(0, n))

        for _ in range(n_static):
            cy = centre(H)
            cx = centre(W)
            self.static.append((cy, cx, float(rng.uniform(0, 2 * math.pi))))
        self.mover_y = centre(H)
        self.mover_x0 = int(rng.integers(0, W))
        self.mover_phi = float(rng.uniform(0, 2 * math.pi))
        self.maxv = (1 << bits) - 1
        self.dtype = np.uint16 if bits > 8 else np.uint8
        r = radius
        yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
        self._disk = (yy * yy + xx * xx) <= r * r

    def _stamp(self, img, cy, cx, value):
        r = self.radius
        ys = np.arange(cy - r, cy + r + 1)
        xs = np.arange(cx - r, cx + r + 1) % self.W
        ok = (ys >= 0) & (ys < self.H)
        sub = self._disk[ok]
        img[np.ix_(ys[ok], xs)] += (sub * value).astype(np.int32)

    def cycle(self, c):
        """The four frames of cycle ``c`` (frames 4c .. 4c+3) as [4][H][W]."""
        out = np.empty((4, self.H, self.W), dtype=self.dtype)
        bank = self.noise.shape[0]
        for j in range(4):
            t = 4 * c + j
            img = self.noise[t % bank].copy()
            for cy, cx, phi in self.static:
                self._stamp(img, cy, cx, int(square_wave(t, phi) * self.amplitude))
            mx = (self.mover_x0 + c) % self.W
            self._stamp(img, self.mover_y, mx, int(square_wave(t, self.mover_phi) * self.amplitude))
            np.clip(img, 0, self.maxv, out=img)
            out[j] = img.astype(self.dtype)
        return out

    def frames(self, c0, n_cycles):
        return np.concatenate([self.cycle(c) for c in range(c0, c0 + n_cycles)], axis=0)


STREAM_SHAPES = ((512, 640), (1024, 1280), (2048, 2048))   # (H, W) of the three cameras


# ---------------------------------------------------------------------------
# Tiles for the learned short-window path: Poisson background, weak ballistic
# modulation inside random rectangles, one random phase per tile.
# ---------------------------------------------------------------------------
def tile_params(seed, n_tiles, H=512, W=512, background=2000.0, ballistic=5e-4,
                smin=16, smax=256, max_rects=5):
    """Per-tile masks and the four per-phase Poisson rates inside/outside the mask.

    Returns dict with ``mask`` uint8 [n][H][W] and ``rates`` float64 [n][2][4]:
    rates[i][0][j] = background (outside), rates[i][1][j] =
    background + ballistic*background*(1 + cos(pi j / 2 + phi_i)) for phase j.
    Also ``phi`` [n].  ``ballistic`` may be a pair (lo, hi): then each tile
    draws its fraction log-uniformly from [lo, hi].
    """
    rng = np.random.default_rng(seed)
    masks = np.zeros((n_tiles, H, W), dtype=np.uint8)
    rates = np.zeros((n_tiles, 2, 4), dtype=np.float64)
    phis = np.zeros(n_tiles)
    for i in range(n_tiles):
        n = int(rng.integers(1, max_rects + 1))
        m, _ = rect_masks(rng, H, W, n, smin, min(smax, H, W))
        masks[i] = m
        phi = float(rng.uniform(0, 2 * math.pi))
        phis[i] = phi
        if isinstance(ballistic, (tuple, list)):
            A = background * math.exp(rng.uniform(math.log(ballistic[0]), math.log(ballistic[1])))
        else:
            A = ballistic * background
        for j in range(4):
            rates[i, 0, j] = background
            rates[i, 1, j] = background + A * (1.0 + math.cos(math.pi * j / 2.0 + phi))
    return dict(mask=masks, rates=rates, phi=phis, background=background, ballistic=ballistic)


class ClutterMotionScene:
    """A camera scene with moving sources and clutter, rendered on a device.

    1024 x 1024 frames with 12-bit Poisson samples, four frames per modulation
    period (frame t has phase t mod 4), of rate

      background 2000
      + 6 point sources: Gaussian spots (sigma 1.5 px) of ballistic amplitude
        20 counts, modulated 20 (1 + cos(pi t / 2 + phi_i + 0.01 c)) (a phase
        drift of 0.01 rad per cycle c = t // 4), moving at U[0, 2] px per cycle
        in random directions (wrapping at the frame edges)
      + 2 clutter spots (sigma 4 px) of amplitude 200 modulated at 1.5 times
        the lock-in frequency, 200 (1 + cos(3 pi t / 4 + psi_j))
      + 2 steady clutter spots (sigma 4 px) of 200 counts
      + an extended disk (radius 64) of ballistic fraction 1e-4 (0.2 counts),
        0.2 (1 + cos(pi t / 2 + phi_d)).

    ``rates(t)`` renders the rate of frame t; ``signal_rates(t)`` only the
    terms modulated at the lock-in frequency (points and disk), the
    noise-free signal the images are judged against; ``frames(c0, n)`` draws
    the Poisson frames of cycles c0 .. c0+n-1 from a seeded device generator.
    """

    N_POINTS, N_CLUTTER_AC, N_CLUTTER_DC = 6, 2, 2

    def __init__(self, seed, H=1024, W=1024, device="cuda", background=2000.0, point_amp=20.0, psf_sigma=1.5,
                 drift=0.01, vmax=2.0, clutter_amp=200.0, clutter_sigma=4.0, disk_r=64, disk_frac=1e-4, bits=12):
        import torch
        self.torch = torch
        rng = np.random.default_rng(seed)
        self.seed, self.H, self.W, self.device, self.bits = seed, H, W, device, bits
        self.background, self.point_amp, self.psf_sigma, self.drift = background, point_amp, psf_sigma, drift
        self.clutter_amp, self.clutter_sigma = clutter_amp, clutter_sigma
        m = 3 * disk_r
        self.p0 = np.stack([rng.uniform(16, H - 16, self.N_POINTS), rng.uniform(16, W - 16, self.N_POINTS)], 1)
        speed = rng.uniform(0, vmax, self.N_POINTS)
        ang = rng.uniform(0, 2 * math.pi, self.N_POINTS)
        self.v = np.stack([speed * np.sin(ang), speed * np.cos(ang)], 1)        # px per cycle (y, x)
        self.phi = rng.uniform(0, 2 * math.pi, self.N_POINTS)
        nc = self.N_CLUTTER_AC + self.N_CLUTTER_DC
        self.clutter = np.stack([rng.uniform(32, H - 32, nc), rng.uniform(32, W - 32, nc)], 1)
        self.psi = rng.uniform(0, 2 * math.pi, self.N_CLUTTER_AC)
        self.disk = (float(rng.uniform(m, H - m)), float(rng.uniform(m, W - m)), disk_r)
        self.phi_d = float(rng.uniform(0, 2 * math.pi))
        self.disk_amp = disk_frac * background
        yy = torch.arange(H, device=device, dtype=torch.float32)[:, None]
        xx = torch.arange(W, device=device, dtype=torch.float32)[None, :]
        self.yy, self.xx = yy, xx
        cy, cx, r = self.disk
        self.disk_mask = (((yy - cy) ** 2 + (xx - cx) ** 2) <= r * r).to(torch.float32)
        cl = torch.zeros((nc, H, W), device=device)
        for j in range(nc):
            cl[j] = torch.exp(-((yy - self.clutter[j, 0]) ** 2 + (xx - self.clutter[j, 1]) ** 2)
                              / (2 * clutter_sigma ** 2))
        self.cl = cl
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(int(seed))

    def point_positions(self, t):
        """(y, x) of the point sources at frame t (wrapped into the frame)."""
        p = self.p0 + self.v * (t / 4.0)
        return np.stack([np.mod(p[:, 0], self.H), np.mod(p[:, 1], self.W)], 1)

    def _spots(self, t):
        torch = self.torch
        pos = self.point_positions(t)
        c = t // 4
        out = torch.zeros((self.H, self.W), device=self.device)
        for i in range(self.N_POINTS):
            dy = torch.remainder(self.yy - float(pos[i, 0]) + self.H / 2, self.H) - self.H / 2
            dx = torch.remainder(self.xx - float(pos[i, 1]) + self.W / 2, self.W) - self.W / 2
            g = torch.exp(-(dy * dy + dx * dx) / (2 * self.psf_sigma ** 2))
            out += g * (self.point_amp * (1.0 + math.cos(math.pi * t / 2 + self.phi[i] + self.drift * c)))
        return out

    def signal_rates(self, t):
        return self._spots(t) + self.disk_mask * (self.disk_amp * (1.0 + math.cos(math.pi * t / 2 + self.phi_d)))

    def rates(self, t):
        lam = self.signal_rates(t) + self.background
        for j in range(self.N_CLUTTER_AC):
            lam += self.cl[j] * (self.clutter_amp * (1.0 + math.cos(3 * math.pi * t / 4 + self.psi[j])))
        for j in range(self.N_CLUTTER_DC):
            lam += self.cl[self.N_CLUTTER_AC + j] * self.clutter_amp
        return lam

    def frames(self, c0, n_cycles):
        """uint16 samples (as a torch int16 tensor [4 n][H][W] on the device)."""
        torch = self.torch
        top = float((1 << self.bits) - 1)
        out = torch.empty((4 * n_cycles, self.H, self.W), dtype=torch.int16, device=self.device)
        for k in range(4 * n_cycles):
            lam = self.rates(4 * c0 + k)
            out[k] = torch.clamp(torch.poisson(lam, generator=self.gen), max=top).to(torch.int32).to(torch.int16)
        return out

    def source_regions(self, t):
        """(name, source mask, surround mask) per source at frame t, as numpy bool
        [H][W]: a 3 x 3 block and its 3-px ring for the spots (points and
        clutter), the disk and the annulus r..3r for the disk (clipped)."""
        H, W = self.H, self.W
        out = []

        def block(cy, cx, half):
            m = np.zeros((H, W), dtype=bool)
            y, x = int(round(cy)) % H, int(round(cx)) % W
            m[max(0, y - half):y + half + 1, max(0, x - half):x + half + 1] = True
            return m

        for i, (cy, cx) in enumerate(self.point_positions(t)):
            src = block(cy, cx, 1)
            out.append(("point%d" % i, src, block(cy, cx, 4) & ~src))
        for j, (cy, cx) in enumerate(self.clutter):
            kind = "clutter_1.5f%d" % j if j < self.N_CLUTTER_AC else "clutter_dc%d" % (j - self.N_CLUTTER_AC)
            src = block(cy, cx, 1)
            out.append((kind, src, block(cy, cx, 4) & ~src))
        cy, cx, r = self.disk
        yy, xx = np.mgrid[0:H, 0:W]
        d2 = (yy - cy) ** 2 + (xx - cx) ** 2
        out.append(("disk", d2 <= r * r, (d2 > r * r) & (d2 <= 9 * r * r)))
        return out


FIG1_FREQS = (20.0, 23.0, 26.0, 29.0)           # Hz, the paper's Fig. 1 modulation frequencies


def fig1_analog(seed, N, X=5.0, n=64, m=8, fs=100.0, freqs=FIG1_FREQS, scale=100.0, pedestal=0.5,
                constant=0.5, polarised=None):
    """Synthetic analog of the paper's numerical example (Methods, numerical
    simulations; Fig. 1): an n x n frame with five non-overlapping m x m
    sources, four with intensity 0.5 + sin(2 pi f_i t_s) and one constant,
    frames at t_s = s / fs for s = 1..N, and a uniform U[0, X] number added
    to every pixel of every frame (diffuse and ambient light).  Samples are
    round(scale * (pedestal + intensity + noise)) as uint16 (the pedestal
    keeps them non-negative; it is constant in time).

    polarised=(f_p, ballistic, depolarised): instead of intensity modulation,
    source 0's light has its linear polarisation rotating at f_p and is seen
    through a fixed analyser: ballistic * cos^2(2 pi f_p t_s) + depolarised / 2
    (modulated at 2 f_p); the other sources are off.

    Returns (frames [N][n][n] uint16, sources [(y0, x0)] of the m x m boxes,
    meta dict)."""
    rng = np.random.default_rng(seed)
    q = n // 8
    boxes = [(q, q), (q, n - q - m), (n - q - m, q), (n - q - m, n - q - m), (n // 2 - m // 2, n // 2 - m // 2)]
    t = np.arange(1, N + 1, dtype=np.float64) / fs
    base = np.full((N, n, n), pedestal)
    for i, (y0, x0) in enumerate(boxes):
        if polarised is not None:
            if i == 0:
                fp, ball, depol = polarised
                inten = ball * np.cos(2 * np.pi * fp * t) ** 2 + depol / 2
            else:
                continue
        elif i < len(freqs):
            inten = 0.5 + np.sin(2 * np.pi * freqs[i] * t)
        else:
            inten = np.full(N, constant)
        base[:, y0:y0 + m, x0:x0 + m] += inten[:, None, None]
    noisy = base + rng.uniform(0.0, X, size=base.shape)
    frames = np.clip(np.rint(scale * noisy), 0, 65535).astype(np.uint16)
    return frames, boxes, dict(fs=fs, freqs=freqs, m=m, n=n, X=X, N=N, scale=scale)
