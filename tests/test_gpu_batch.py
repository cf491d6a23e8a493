"""GPU parity of the batch path (qld_accumulate with per-frame statistics,
qld_amplitude, dft_bin_baseline) against the CPU oracle, through the C ABI.

Bar: I/Q and the statistics bit-exact; amplitude within 2 ulp of float32 of
the double-precision oracle; the DFT within (N + 2) 2^-24 sum|x| per component.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1511_03390_amd as qld
import scenes
from tests.gpu_util import amp_ulps, need_gpu, say, to_dev, to_host_u16

pytestmark = pytest.mark.gpu


def run_lockin(frames_np, phase0=0, bits=None, pitch_view=None):
    dev = to_dev(frames_np)
    if pitch_view is not None:
        dev = pitch_view(dev)
    I, Q, amp, fsum, fsat = qld.lockin(dev, phase0=phase0, bits=bits, stats=True)
    torch.cuda.synchronize()
    return I.cpu().numpy(), Q.cpu().numpy(), amp.cpu().numpy(), fsum.cpu().numpy(), fsat.cpu().numpy()


def check_against_oracle(frames_host_view, I, Q, amp, fsum, fsat, phase0, bits):
    oI, oQ = oracle.qld(frames_host_view, phase0)
    assert np.array_equal(I.astype(np.int64), oI), "I differs"
    assert np.array_equal(Q.astype(np.int64), oQ), "Q differs"
    s, n = oracle.frame_stats(frames_host_view, bits)
    assert np.array_equal(fsum.astype(np.uint64), s), "frame sums differ"
    assert np.array_equal(fsat.astype(np.uint32), n), "saturation counts differ"
    oa = oracle.amplitude(oI, oQ)
    u = amp_ulps(amp, oa)
    assert u.max() <= 2.0, u.max()
    return float(u.max())


def test_small_disk_scene_u8():
    need_gpu()
    st = scenes.disk_scene_u8()
    say("disk scene u8", st.frames.shape)
    I, Q, amp, fsum, fsat = run_lockin(st.frames, bits=8)
    check_against_oracle(st.frames, I, Q, amp, fsum, fsat, 0, 8)
    # The modulated disk stands out: square-wave closed form 2 sqrt(2) M A = 181.02 minus noise.
    m = st.meta["mask"]
    assert amp[m].mean() > 3 * amp[~m].mean()


CASES = [
    # (dtype, T, H, W, pitch_extra, phase0, bits, misalign)
    (np.uint16, 64, 17, 33, 0, 0, 12, 0),
    (np.uint16, 67, 5, 8, 8, 1, 12, 0),
    (np.uint16, 5, 3, 1000, 24, 3, 16, 0),
    (np.uint16, 1, 1, 1, 0, 0, 16, 0),
    (np.uint16, 2, 9, 7, 0, 2, 16, 1),
    (np.uint16, 3, 300, 257, 0, 7, 12, 0),
    (np.uint16, 4096, 16, 16, 0, 0, 12, 0),      # frame axis split over many work-groups
    (np.uint16, 1029, 40, 64, 0, -1, 12, 0),
    (np.uint8, 64, 64, 64, 0, 0, 8, 0),
    (np.uint8, 33, 7, 31, 1, 1, 8, 0),
    (np.uint8, 2000, 8, 48, 16, 2, 8, 0),
    (np.uint8, 9, 13, 17, 0, 0, 8, 3),
    # More tiles than work-groups, taken two per unit (wide tiles): u8 (16
    # pixels per lane, 550 tiles), and u16 with padded rows (600 tiles).
    (np.uint8, 130, 1100, 2048, 0, 1, 8, 0),
    (np.uint16, 134, 600, 2048, 8, 3, 12, 0),
    # 16-bit data without the packed partials (bits 16): two tiles per unit
    # (600 tiles), then 1100 tiles = 550 wide tiles, one round of 512 and the
    # other 38 split two ways over the frames.
    (np.uint16, 40, 600, 2048, 0, 2, 16, 0),
    (np.uint16, 130, 1100, 2048, 0, 1, 16, 0),
    # u8, 1050 tiles two per unit: one round of 512 wide tiles, the other 13
    # split two ways over the frames, ragged last cycle.
    (np.uint8, 130, 2100, 2048, 0, 3, 8, 0),
]


@pytest.mark.parametrize("dt,T,H,W,pextra,phase0,bits,mis", CASES)
def test_random_shapes(dt, T, H, W, pextra, phase0, bits, mis):
    need_gpu()
    rng = np.random.default_rng(1000 + T * 7 + W)
    say("shape case", dt.__name__, T, H, W, pextra, phase0, bits, mis)
    pitch = W + pextra + mis
    buf, _ = scenes.random_stack(rng, T, H, pitch, dt, bits=bits)
    # Include saturated samples so the count is exercised.
    buf[:, ::3, ::5] = (1 << bits) - 1
    view_host = buf[:, :, mis:mis + W]
    dev_full = to_dev(buf)
    dev = dev_full[:, :, mis:mis + W]
    I, Q, amp, fsum, fsat = qld.lockin(dev, phase0=phase0, bits=bits, stats=True)
    torch.cuda.synchronize()
    check_against_oracle(view_host, I.cpu().numpy(), Q.cpu().numpy(), amp.cpu().numpy(), fsum.cpu().numpy(),
                         fsat.cpu().numpy(), phase0, bits)


def test_accumulate_onto_running_sums_with_split_tail():
    # 600 tiles: the first 512 add into I/Q in the kernel, the split tail in
    # the partials' reduction; accumulating a stack onto running sums (two
    # chunks with the phase carried over, on top of garbage-free but non-zero
    # I/Q) equals the oracle's sums plus the starting values.
    need_gpu()
    rng = np.random.default_rng(29)
    T, H, W = 258, 600, 2048
    f = rng.integers(0, 4096, size=(T, H, W)).astype(np.uint16)
    dev = to_dev(f)
    I0 = rng.integers(-10 ** 6, 10 ** 6, size=(H, W)).astype(np.int32)
    Q0 = rng.integers(-10 ** 6, 10 ** 6, size=(H, W)).astype(np.int32)
    I = torch.from_numpy(I0).cuda()
    Q = torch.from_numpy(Q0).cuda()
    fsum = torch.zeros(T, dtype=torch.int64, device="cuda")
    fsat = torch.zeros(T, dtype=torch.int32, device="cuda")
    qld.accumulate(dev[:130], I, Q, 2, 12, fsum[:130], fsat[:130])
    qld.accumulate(dev[130:], I, Q, 2 + 130, 12, fsum[130:], fsat[130:])
    torch.cuda.synchronize()
    oI, oQ = oracle.qld(f, 2)
    assert np.array_equal(I.cpu().numpy().astype(np.int64), oI + I0), "I differs"
    assert np.array_equal(Q.cpu().numpy().astype(np.int64), oQ + Q0), "Q differs"
    s, n = oracle.frame_stats(f, 12)
    assert np.array_equal(fsum.cpu().numpy().astype(np.uint64), s)
    assert np.array_equal(fsat.cpu().numpy().astype(np.uint32), n)


def test_chunked_accumulation_equals_whole():
    need_gpu()
    rng = np.random.default_rng(3)
    f = rng.integers(0, 4096, size=(150, 21, 40)).astype(np.uint16)
    dev = to_dev(f)
    I = torch.zeros((21, 40), dtype=torch.int32, device="cuda")
    Q = torch.zeros_like(I)
    done = 0
    for n in (1, 6, 37, 50, 56):
        qld.accumulate(dev[done:done + n], I, Q, phase0=done, bits=12)
        done += n
    torch.cuda.synchronize()
    oI, oQ = oracle.qld(f)
    assert np.array_equal(I.cpu().numpy(), oI) and np.array_equal(Q.cpu().numpy(), oQ)


def test_full_range_16bit_and_overflow_edge():
    need_gpu()
    M = 32768
    f = np.zeros((4 * M, 1, 8), dtype=np.uint16)
    f[0::4] = 65535
    f[1::4, :, ::2] = 65535
    dev = to_dev(f)
    I, Q, amp = qld.lockin(dev, bits=16)
    torch.cuda.synchronize()
    assert (I.cpu().numpy() == 65535 * M).all()
    assert (Q.cpu().numpy()[0, ::2] == 65535 * M).all() and (Q.cpu().numpy()[0, 1::2] == 0).all()
    with pytest.raises(qld.QldError) as e:
        qld.lockin(to_dev(np.zeros((4 * M + 1, 1, 8), np.uint16)), bits=16)
    assert e.value.status == qld.E_OVERFLOW


@pytest.mark.parametrize("T,H,W,bits,phase0", [(64, 17, 40, 12, 1), (4096, 16, 16, 12, 0), (9, 5, 1003, 16, 3),
                                               (1024, 64, 64, 12, 2),
                                               # more pixel tiles than work-groups: 550 tiles, two
                                               # per unit (275 wide tiles, one round, unsplit)
                                               (64, 1100, 1024, 12, 3),
                                               # 520 tiles plus a 4-column scalar tail, ragged
                                               # last cycle
                                               (130, 520, 2052, 12, 1),
                                               # 300 tiles split in two: 608 units on 512
                                               # work-groups (some take two units)
                                               (256, 300, 2048, 12, 2),
                                               # 600 tiles, two per unit
                                               (262, 600, 2048, 12, 1),
                                               # 2048 tiles, four per unit: one round of 512
                                               # wide tiles
                                               (64, 2048, 2048, 12, 0),
                                               # 2100 tiles, four per unit: one round of 512
                                               # wide tiles, the other 13 split 2 ways over
                                               # the frames (partials from row 2048 on),
                                               # ragged last cycle
                                               (130, 2100, 2048, 12, 1)])
def test_lockin_image_overwrites_and_matches_accumulate(T, H, W, bits, phase0):
    """qld_lockin_image (one pass: I/Q, amplitude and statistics overwritten)
    on garbage-filled outputs equals clearing them, qld_accumulate and
    qld_amplitude, and the oracle; frame-split grids and row tails included."""
    need_gpu()
    rng = np.random.default_rng(T + H + W)
    f = rng.integers(0, 1 << bits, size=(T, H, W)).astype(np.uint16)
    f[:, ::7, ::3] = (1 << bits) - 1
    dev = to_dev(f)
    I = torch.full((H, W), 123456, dtype=torch.int32, device="cuda")
    Q = torch.full_like(I, -98765)
    amp = torch.full((H, W), 7.5, dtype=torch.float32, device="cuda")
    fsum = torch.full((T,), 99, dtype=torch.int64, device="cuda")
    fsat = torch.full((T,), 77, dtype=torch.int32, device="cuda")
    qld.lockin_image(dev, I, Q, amp, phase0=phase0, bits=bits, frame_sum=fsum, frame_sat=fsat)
    I2 = torch.zeros_like(I)
    Q2 = torch.zeros_like(Q)
    s2 = torch.zeros_like(fsum)
    c2 = torch.zeros_like(fsat)
    a2 = torch.empty_like(amp)
    qld.accumulate(dev, I2, Q2, phase0, bits, s2, c2)
    qld.amplitude(I2, Q2, a2)
    torch.cuda.synchronize()
    for x, y in ((I, I2), (Q, Q2), (amp, a2), (fsum, s2), (fsat, c2)):
        assert torch.equal(x, y)
    check_against_oracle(f, I.cpu().numpy(), Q.cpu().numpy(), amp.cpu().numpy(), fsum.cpu().numpy(),
                         fsat.cpu().numpy(), phase0, bits)
    with pytest.raises(qld.QldError) as e:
        qld.lockin_image(dev[:0], I, Q, amp, bits=bits)
    assert e.value.status == qld.E_SHAPE


def test_statistics_over_odd_flush_counts_and_grid_rounds():
    """Per-frame statistics when each persistent-grid unit ends on an odd
    number of statistics flushes and work-groups take several units: 300
    tiles split 2 ways over 808 frames make 608 units on 512 work-groups
    (96 of them take two), each unit 404 frames, 7 flushes of up to 64
    frames.  The sums and counts stay exact across the units of a
    work-group."""
    need_gpu()
    rng = np.random.default_rng(808)
    T, H, W, bits = 808, 300, 2048, 12
    f = rng.integers(0, 1 << bits, size=(T, H, W), dtype=np.uint16)
    f[:, ::9, ::4] = (1 << bits) - 1
    say("statistics case", T, H, W)
    dev = to_dev(f)
    I, Q, amp, fsum, fsat = qld.lockin(dev, phase0=1, bits=bits, stats=True)
    torch.cuda.synchronize()
    check_against_oracle(f, I.cpu().numpy(), Q.cpu().numpy(), amp.cpu().numpy(), fsum.cpu().numpy(),
                         fsat.cpu().numpy(), 1, bits)


def test_hinted_frame_stride_gives_the_same_image():
    # A stack laid out with qld_frame_stride_hint (gaps between frames) gives
    # the same I/Q, amplitude and statistics as the dense layout.
    need_gpu()
    T, H, W = 64, 256, 256
    fs = qld.frame_stride_hint(H, W)
    assert fs > H * W
    rng = np.random.default_rng(11)
    f = rng.integers(0, 4096, size=(T, H, W)).astype(np.uint16)
    dense = to_dev(f)
    padded = torch.full((T * fs,), -1, dtype=torch.int16, device="cuda").as_strided((T, H, W), (fs, W, 1))
    padded.copy_(dense)
    outs = []
    for stack in (dense, padded):
        I = torch.empty((H, W), dtype=torch.int32, device="cuda")
        Q = torch.empty_like(I)
        amp = torch.empty((H, W), dtype=torch.float32, device="cuda")
        fsum = torch.empty(T, dtype=torch.int64, device="cuda")
        fsat = torch.empty(T, dtype=torch.int32, device="cuda")
        qld.lockin_image(stack, I, Q, amp, 1, 12, fsum, fsat)
        outs.append([x.cpu() for x in (I, Q, amp, fsum, fsat)])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    I, Q, amp, fsum, fsat = (x.numpy() for x in outs[1])
    check_against_oracle(f, I, Q, amp, fsum, fsat, 1, 12)


def test_read_probe_xor_of_every_word():
    need_gpu()
    rng = np.random.default_rng(3)
    for nbytes in (16, 4096 + 48, (3 << 20) + 16 * 7):
        h = rng.integers(0, 256, size=nbytes, dtype=np.uint8)
        dev = torch.from_numpy(h).cuda()
        out = qld.read_probe(dev)
        torch.cuda.synchronize()
        ref = np.bitwise_xor.reduce(h.view(np.uint64))
        assert int(out.cpu().numpy().view(np.uint64)[0]) == int(ref), nbytes


def test_amplitude_extremes():
    need_gpu()
    rng = np.random.default_rng(4)
    I = np.concatenate([np.array([0, 1, -1, 3, 2 ** 31 - 1, -(2 ** 31 - 1), 46341, 2 ** 30, 5], np.int32),
                        rng.integers(-2 ** 31 + 1, 2 ** 31 - 1, 100000, dtype=np.int64).astype(np.int32)])
    Q = np.concatenate([np.array([0, 0, 1, 4, 2 ** 31 - 1, 2 ** 31 - 1, 46341, -2 ** 30, 12], np.int32),
                        rng.integers(-2 ** 31 + 1, 2 ** 31 - 1, 100000, dtype=np.int64).astype(np.int32)])
    dI, dQ = torch.from_numpy(I).cuda(), torch.from_numpy(Q).cuda()
    amp = torch.empty(len(I), dtype=torch.float32, device="cuda")
    qld.amplitude(dI, dQ, amp)
    a = amp.cpu().numpy()
    oa = oracle.amplitude(I.astype(np.int64), Q.astype(np.int64))
    u = amp_ulps(a, oa)
    say("amplitude max ulp", u.max())
    assert u.max() <= 2.0
    assert a[0] == 0 and a[1] == 1 and a[3] == 5 and a[8] == 13


def dft_bound(frames_host, N):
    x = frames_host.astype(np.float64)
    return (N + 2) * 2.0 ** -24 * np.abs(x).sum(axis=0)


def bank_fast_path(dev):
    """The bank's staged paths take 16-bit stacks with 16-byte aligned base and
    W, row pitch and frame stride multiples of 8 elements."""
    T, H, W = dev.shape
    return (dev.element_size() == 2 and dev.data_ptr() % 16 == 0 and W % 8 == 0 and dev.stride(1) % 8 == 0
            and dev.stride(0) % 8 == 0)


def bank_bf16_freqs(F, fast):
    """Which frequencies the bf16 path computes: frequencies go in groups of
    32, and a staged group of more than 8 takes the bf16 path."""
    return np.array([fast and min(32, F - 32 * (f // 32)) > 8 for f in range(F)])


def bank_bound(frames_host, N, bf16):
    """Per-pixel error bound of the bank against the exact lock-in, [F][H][W].
    Float paths: float products and sums, as the DFT.  bf16 path: each frame
    gives six exact products xh b_i, xl b_i (sum of magnitudes <= 1.01 x |Bf|,
    Bf the float twiddle), 6N terms summed in fp32 ((6N - 1) u), plus the
    split's and the float table's rounding (2 u), u = 2^-24."""
    x = np.abs(frames_host.astype(np.float64)).sum(axis=0)
    k = np.where(np.asarray(bf16), (6 * N + 2) * 1.01, N + 2)
    return k[:, None, None] * 2.0 ** -24 * x[None]


@pytest.mark.parametrize("T,H,W,k,dt", [(64, 33, 40, 16, np.uint16), (1024, 16, 64, 256, np.uint16),
                                        (37, 5, 9, 3, np.uint8), (300, 4, 24, -5, np.uint8),
                                        (2048, 3, 20, 777, np.uint16)])
def test_dft_bin_baseline_f64(T, H, W, k, dt):
    """The double-precision DFT against the oracle's double DFT.  GPU: one
    rounding per fused multiply-add, twiddles from sincospi of the exact
    integer angle: within (N + 8) 2^-53 sum|x| of the exact value.  Oracle:
    a rounded product and a rounded sum per term, twiddles from cos/sin of
    2 pi r / N formed in double (about 20 units of 2^-53): within
    (2N + 24) 2^-53 sum|x|.  So they agree within (3N + 48) 2^-53 sum|x|."""
    need_gpu()
    rng = np.random.default_rng(T + W)
    bits = 12 if dt == np.uint16 else 8
    f = rng.integers(0, 1 << bits, size=(T, H, W)).astype(dt)
    re = torch.empty((H, W), dtype=torch.float64, device="cuda")
    im = torch.empty_like(re)
    qld.dft_bin_baseline_f64(to_dev(f), k, re, im, bits=bits)
    torch.cuda.synchronize()
    X = oracle.dft_bin(f, k)
    bound = (3 * T + 48) * 2.0 ** -53 * np.abs(f.astype(np.float64)).sum(axis=0)
    er, ei = np.abs(re.cpu().numpy() - X.real), np.abs(im.cpu().numpy() - X.imag)
    say("dft f64 max err", er.max(), ei.max(), "bound", bound.min())
    assert (er <= bound).all() and (ei <= bound).all()
    # Orders of magnitude closer than the float path can be.
    assert er.max() <= 2.0 ** -24 * np.abs(f.astype(np.float64)).sum(axis=0).min()


@pytest.mark.parametrize("T,H,W,k,dt", [(64, 33, 40, 16, np.uint16), (1024, 16, 64, 256, np.uint16),
                                        (37, 5, 9, 3, np.uint8), (256, 8, 8, 7, np.uint16),
                                        (300, 4, 24, -5, np.uint8)])
def test_dft_bin_baseline(T, H, W, k, dt):
    need_gpu()
    rng = np.random.default_rng(T + W)
    bits = 12 if dt == np.uint16 else 8
    f = rng.integers(0, (1 << bits), size=(T, H, W)).astype(dt)
    dev = to_dev(f)
    re = torch.empty((H, W), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    qld.dft_bin_baseline(dev, k, re, im, bits=bits)
    torch.cuda.synchronize()
    X = oracle.dft_bin(f, k)
    bound = dft_bound(f, T)
    err_r = np.abs(re.cpu().numpy() - X.real)
    err_i = np.abs(im.cpu().numpy() - X.imag)
    say("dft max err", err_r.max(), err_i.max(), "bound", bound.min())
    assert (err_r <= bound).all() and (err_i <= bound).all()
    if k % T == T // 4 and T % 4 == 0:
        oI, oQ = oracle.qld(f)
        assert np.abs(re.cpu().numpy() - oI).max() <= bound.max()
        assert np.abs(im.cpu().numpy() + oQ).max() <= bound.max()


@pytest.mark.parametrize("T,H,W,p,q,t0,dt", [(64, 33, 40, 1, 4, 3, np.uint16), (200, 16, 64, 3, 20, 0, np.uint16),
                                              (37, 5, 9, 7, 11, 5, np.uint8), (300, 4, 24, -2, 9, 1, np.uint8),
                                              (1024, 8, 72, 23, 100, 17, np.uint16)])
def test_lockin_ratio(T, H, W, p, q, t0, dt):
    """General-ratio lock-in against the oracle (double, exact angle reduction)
    within the float accumulation bound; p/q = 1/4 equals the integer QLD."""
    need_gpu()
    rng = np.random.default_rng(T + W + q)
    bits = 12 if dt == np.uint16 else 8
    f = rng.integers(0, (1 << bits), size=(T, H, W)).astype(dt)
    re = torch.empty((H, W), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    qld.lockin_ratio(to_dev(f), p, q, re, im, t0=t0, bits=bits)
    torch.cuda.synchronize()
    X = oracle.lockin_ratio(f, p, q, t0)
    bound = dft_bound(f, T)
    err_r = np.abs(re.cpu().numpy() - X.real)
    err_i = np.abs(im.cpu().numpy() - X.imag)
    say("lock-in ratio", p, q, "max err", err_r.max(), err_i.max(), "bound", bound.min())
    assert (err_r <= bound).all() and (err_i <= bound).all()
    if (p, q) == (1, 4):
        oI, oQ = oracle.qld(f, t0 % 4)
        assert np.abs(re.cpu().numpy() - oI).max() <= bound.max()
        assert np.abs(im.cpu().numpy() + oQ).max() <= bound.max()


def test_lockin_ratio_rejects_another_frequency():
    """Wrong-frequency rejection: a source at 3/20 of the frame rate next to one
    at 7/20; each lock-in sees its own source (A T / 2) and not the other."""
    need_gpu()
    T, H, W = 400, 8, 32
    t = np.arange(T)[:, None, None]
    x = np.arange(W)[None, None, :]
    left = x < W // 2
    sig = 1000 + np.where(left, 200 * np.cos(2 * np.pi * 3 * t / 20), 120 * np.cos(2 * np.pi * 7 * t / 20 + 0.4))
    f = np.broadcast_to(np.rint(sig), (T, H, W)).astype(np.uint16)
    re = torch.empty((H, W), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    amp = {}
    for p in (3, 7):
        qld.lockin_ratio(to_dev(f), p, 20, re, im, bits=12)
        torch.cuda.synchronize()
        amp[p] = np.hypot(re.cpu().numpy(), im.cpu().numpy())
    resid = np.abs(np.rint(sig) - sig).sum(axis=0)              # sample rounding
    tol = resid + dft_bound(f, T)
    lmask = np.broadcast_to(left[0], (H, W))
    assert np.all(np.abs(amp[3][lmask] - 200 * T / 2) <= tol[lmask]) and np.all(amp[3][~lmask] <= tol[~lmask])
    assert np.all(np.abs(amp[7][~lmask] - 120 * T / 2) <= tol[~lmask]) and np.all(amp[7][lmask] <= tol[lmask])


@pytest.mark.parametrize("T,H,W,F,q,t0,dt", [(64, 9, 40, 1, 64, 0, np.uint16), (100, 13, 37, 5, 100, 3, np.uint16),
                                              (77, 5, 130, 17, 20, 1, np.uint8), (256, 16, 64, 32, 256, 0, np.uint16),
                                              (33, 3, 70, 40, 33, 7, np.uint16), (45, 7, 24, 33, 45, 2, np.uint16),
                                              (70, 11, 48, 9, 35, 5, np.uint16), (50, 6, 32, 20, 50, 1, np.uint16),
                                              (1, 8, 64, 32, 97, 5, np.uint16), (2, 4, 40, 12, 13, 0, np.uint16)])
def test_lockin_bank(T, H, W, F, q, t0, dt):
    """Bank of F lock-ins against the oracle's lock-in at each frequency, within
    the bound of the path each group of 32 frequencies takes.  With one or two
    frames the bf16 bound (6N + 2)·1.01·2^-24·x is far below what dropping a
    twiddle's third bf16 term would cost (up to 2^-16 x)."""
    need_gpu()
    rng = np.random.default_rng(T * F + W)
    bits = 12 if dt == np.uint16 else 8
    f = rng.integers(0, (1 << bits), size=(T, H, W)).astype(dt)
    ps = [int(v) for v in rng.integers(-q, 2 * q, size=F)]
    dev = to_dev(f)
    if W == 48:
        # Padded rows and frames (pitch 56, frame stride from the hint): the 16-byte tile path.
        fs = qld.frame_stride_hint(H, W, row_pitch=56)
        buf = torch.full((T * fs,), 0x5A5A, dtype=torch.int16, device="cuda")
        view = buf.as_strided((T, H, W), (fs, 56, 1))
        view.copy_(dev)
        dev = view
    re, im = qld.lockin_bank(dev, ps, q, t0=t0, bits=bits)
    torch.cuda.synchronize()
    X = oracle.lockin_bank(f, ps, q, t0)
    fast = bank_fast_path(dev)
    assert fast == (dt == np.uint16 and W % 8 == 0)
    bf16 = bank_bf16_freqs(F, fast)
    bound = bank_bound(f, T, bf16)
    err_r = np.abs(re.cpu().numpy() - X.real)
    err_i = np.abs(im.cpu().numpy() - X.imag)
    say("bank F", F, "fast", fast, "bf16 groups", int(bf16.sum()), "max err", err_r.max(), err_i.max(), "bound", bound.min(),
        "max err / float bound", max((err_r / dft_bound(f, T)[None]).max(), (err_i / dft_bound(f, T)[None]).max()))
    assert (err_r <= bound).all() and (err_i <= bound).all()


def test_lockin_bank_separates_four_sources():
    """Four sources modulated at 20, 23, 26 and 29 Hz seen at 100 frames/s (the
    paper's Fig. 1 frequencies): over whole beat periods each image of the bank
    shows its own source only."""
    need_gpu()
    T, H, W = 500, 4, 64
    t = np.arange(T)[:, None, None]
    x = np.arange(W)[None, None, :]
    freqs = [20, 23, 26, 29]
    sig = np.full((T, 1, W), 1500.0)
    for j, fq in enumerate(freqs):
        sig = sig + np.where(x // 16 == j, 300 * np.cos(2 * np.pi * fq * t / 100 + 0.3 * j), 0.0)
    f = np.broadcast_to(np.rint(sig), (T, H, W)).astype(np.uint16)
    re, im = qld.lockin_bank(to_dev(f), freqs, 100, bits=12)
    torch.cuda.synchronize()
    amp = np.hypot(re.cpu().numpy(), im.cpu().numpy())
    tol = np.abs(np.rint(sig) - sig).sum(axis=0) + bank_bound(f, T, bank_bf16_freqs(4, True)).max(axis=0)
    for j in range(4):
        own = np.broadcast_to((x // 16 == j)[0], (H, W))
        assert np.all(np.abs(amp[j][own] - 300 * T / 2) <= tol[own]), j
        assert np.all(amp[j][~own] <= tol[~own]), j


def test_full_size_diffuse_scene_sampled():
    """1024 x 1024 uint16 (12-bit), 1024 frames in the benchmark's layout (frame
    stride from the hint) and launches (qld_lockin_image into uninitialised
    outputs, the single-bin DFT, the 32-frequency bank at bins 240..271):
    sampled pixels checked by the oracle one by one; statistics against
    torch's sums."""
    need_gpu()
    fs = qld.frame_stride_hint(1024, 1024)
    st = scenes.diffuse_scene_u16(device="cuda", frame_stride=fs)
    frames = st.frames
    assert frames.stride(0) == fs
    say("full-size stack", tuple(frames.shape), "frame stride", fs)
    I = torch.empty((1024, 1024), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    amp = torch.empty((1024, 1024), dtype=torch.float32, device="cuda")
    fsum = torch.empty(1024, dtype=torch.int64, device="cuda")
    fsat = torch.empty(1024, dtype=torch.int32, device="cuda")
    qld.lockin_image(frames, I, Q, amp, 0, 12, fsum, fsat)
    re = torch.empty((1024, 1024), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    qld.dft_bin_baseline(frames, 256, re, im, bits=12)
    ps = list(range(240, 272))
    bre = torch.empty((32, 1024, 1024), dtype=torch.float32, device="cuda")
    bim = torch.empty_like(bre)
    qld.lockin_bank(frames, ps, 1024, bre, bim, bits=12)
    assert bank_fast_path(frames)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    ys = np.concatenate([[0, 1023, 511], rng.integers(0, 1024, 61)])
    xs = np.concatenate([[0, 1023, 512], rng.integers(0, 1024, 61)])
    sub = frames[:, torch.from_numpy(ys).cuda(), :][:, :, torch.from_numpy(xs).cuda()]
    sub_h = to_host_u16(sub)                 # [T][64][64], the sampled pixels' series
    oI, oQ = oracle.qld(sub_h)
    Ih, Qh, ah = I.cpu().numpy(), Q.cpu().numpy(), amp.cpu().numpy()
    assert np.array_equal(Ih[np.ix_(ys, xs)], oI) and np.array_equal(Qh[np.ix_(ys, xs)], oQ)
    assert amp_ulps(ah[np.ix_(ys, xs)], oracle.amplitude(oI, oQ)).max() <= 2.0
    X = oracle.dft_bin(sub_h, 256)
    bound = dft_bound(sub_h, 1024)
    assert (np.abs(re.cpu().numpy()[np.ix_(ys, xs)] - X.real) <= bound).all()
    assert (np.abs(im.cpu().numpy()[np.ix_(ys, xs)] - X.imag) <= bound).all()
    XB = oracle.lockin_bank(sub_h, ps, 1024)                    # [32][64][64]
    bb = bank_bound(sub_h, 1024, bank_bf16_freqs(32, True))
    gre = bre.cpu().numpy()[:, ys][:, :, xs]
    gim = bim.cpu().numpy()[:, ys][:, :, xs]
    say("bank max err", np.abs(gre - XB.real).max(), "bound", bb.min())
    assert (np.abs(gre - XB.real) <= bb).all() and (np.abs(gim - XB.imag) <= bb).all()
    del bre, bim
    # Per-frame statistics of the whole stack against torch's own reductions.
    ref_sum = frames.to(torch.int64).sum(dim=(1, 2))
    ref_sat = (frames == 4095).sum(dim=(1, 2))
    assert torch.equal(fsum, ref_sum) and torch.equal(fsat.to(torch.int64), ref_sat.to(torch.int64))
    # Drift closed form: the linear ambient ramp leaves I = Q = -2 b M on average
    # (b = 100/1023 per frame, M = 256) -- about -50 outside the modulated mask.
    mask = torch.from_numpy(st.meta["mask"]).cuda()
    mI = I[~mask].double().mean().item()
    assert abs(mI - (-2 * (100 / 1023) * 256)) < 6.0   # ~5 sigma of the mean of ~1e6 noisy pixels
