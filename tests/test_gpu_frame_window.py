"""GPU parity of the per-frame sliding window (an image for every frame)
against the oracle's brute-force per-frame window, which re-sums the stored
frames and never subtracts.

Bar: I/Q bit-exact after every frame, amplitude within 2 ulp of float32,
warm flag and counters as defined; resets with a new phase; agreement with
the cycle window at cycle-aligned frames.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1511_03390_amd as qld
from tests.gpu_util import amp_ulps, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def run(frames, H, W, M, bits, dt, phase0=0, resets=None):
    fw = qld.FrameWindow(H, W, M, phase0=phase0, dtype=torch.uint8 if dt == np.uint8 else torch.int16, bits=bits)
    I = torch.empty((H, W), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    amp = torch.empty((H, W), dtype=torch.float32, device="cuda")
    out = []
    since = 0
    for f, fr in enumerate(frames):
        if resets and f in resets:
            fw.reset(resets[f])
            since = 0
        warm = fw.update(to_dev(fr), I, Q, amp)
        since += 1
        torch.cuda.synchronize()
        assert warm == (1 if since >= 4 * M else 0)
        assert fw.info() == (min(since, 4 * M), since)
        out.append((I.cpu().numpy().copy(), Q.cpu().numpy().copy(), amp.cpu().numpy().copy()))
    fw.close()
    return out


@pytest.mark.parametrize("H,W,M,bits,dt,n,phase0", [(9, 13, 2, 12, np.uint16, 21, 0), (7, 40, 1, 8, np.uint8, 13, 3),
                                                    (32, 64, 3, 16, np.uint16, 30, 1), (1, 1, 1, 12, np.uint16, 9, 2),
                                                    (130, 257, 2, 12, np.uint16, 11, 0)])
def test_frame_window_matches_brute_force_every_frame(H, W, M, bits, dt, n, phase0):
    need_gpu()
    say("frame window", H, W, M, bits, n, phase0)
    rng = np.random.default_rng(H * W + M + phase0)
    frames = [rng.integers(0, 1 << bits, size=(H, W)).astype(dt) for _ in range(n)]
    got = run(frames, H, W, M, bits, dt, phase0)
    for f, (oI, oQ, nin) in enumerate(oracle.frame_window_series(frames, M, phase0)):
        I, Q, amp = got[f]
        assert np.array_equal(I, oI) and np.array_equal(Q, oQ), f
        assert amp_ulps(amp, oracle.amplitude(oI, oQ)).max() <= 2.0, f


@pytest.mark.parametrize("H,W,dt,bits", [(16, 64, np.uint16, 12), (6, 40, np.uint8, 8), (5, 13, np.uint16, 12)])
def test_frame_window_outputs_on_some_frames_only(H, W, dt, bits):
    """Updates without outputs keep only the quadrature that changes; the
    images asked for later still equal the oracle's re-summed window (vector
    and per-pixel kernels)."""
    need_gpu()
    M, n = 2, 29
    rng = np.random.default_rng(H + W)
    frames = [rng.integers(0, 1 << bits, size=(H, W)).astype(dt) for _ in range(n)]
    fw = qld.FrameWindow(H, W, M, phase0=1, dtype=torch.uint8 if dt == np.uint8 else torch.int16, bits=bits)
    I = torch.empty((H, W), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    amp = torch.empty((H, W), dtype=torch.float32, device="cuda")
    want = {f for f in range(n) if f % 5 == 4 or f == n - 1}
    got = {}
    for f, fr in enumerate(frames):
        if f in want:
            fw.update(to_dev(fr), I, Q, amp)
            torch.cuda.synchronize()
            got[f] = (I.cpu().numpy().copy(), Q.cpu().numpy().copy(), amp.cpu().numpy().copy())
        elif f % 5 == 2:
            fw.update(to_dev(fr), None, None, amp)        # the image only
        else:
            fw.update(to_dev(fr))                          # no output at all
    fw.close()
    for f, (oI, oQ, _) in enumerate(oracle.frame_window_series(frames, M, 1)):
        if f in got:
            assert np.array_equal(got[f][0], oI) and np.array_equal(got[f][1], oQ), f
            assert amp_ulps(got[f][2], oracle.amplitude(oI, oQ)).max() <= 2.0, f


def test_frame_window_reset_and_cycle_alignment():
    need_gpu()
    H, W, M = 12, 20, 2
    rng = np.random.default_rng(5)
    frames = [rng.integers(0, 4096, size=(H, W)).astype(np.uint16) for _ in range(26)]
    resets = {10: 3}
    got = run(frames, H, W, M, 12, np.uint16, 0, resets)
    for f, (oI, oQ, _) in enumerate(oracle.frame_window_series(frames, M, 0, resets)):
        assert np.array_equal(got[f][0], oI) and np.array_equal(got[f][1], oQ), f
    # Without resets, at frames that end a cycle the per-frame window equals
    # the cycle window of the library over the same cycles.
    got = run(frames[:24], H, W, M, 12, np.uint16, 0)
    win = qld.Window(H, W, M, bits=12)
    I = torch.empty((H, W), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    for k in range(6):
        win.update(to_dev(np.stack(frames[4 * k:4 * k + 4])), I, Q)
        torch.cuda.synchronize()
        assert np.array_equal(I.cpu().numpy(), got[4 * k + 3][0]) and np.array_equal(Q.cpu().numpy(), got[4 * k + 3][1])
    win.close()


def test_frame_window_steady_amplitude_of_a_sinusoid():
    # Once full, the window always holds M whole periods: a pure 4-frame
    # sinusoid gives the same amplitude after every frame, 2 M (a^2+b^2)^(1/2).
    need_gpu()
    H, W, M = 16, 24, 4
    a, b, c = 30, -40, 2000
    per = [c + a, c + b, c - a, c - b]
    frames = [np.full((H, W), per[t % 4], dtype=np.uint16) for t in range(40)]
    got = run(frames, H, W, M, 12, np.uint16, 0)
    for f in range(4 * M - 1, 40):
        assert np.all(got[f][2] == np.float32(2 * M * 50.0)), f


def test_frame_window_arguments():
    need_gpu()
    with pytest.raises(qld.QldError) as e:
        qld.FrameWindow(8, 8, 0)
    assert e.value.status == qld.E_INVAL
    with pytest.raises(qld.QldError) as e:
        qld.FrameWindow(8, 8, 40000, bits=16)
    assert e.value.status == qld.E_OVERFLOW
    fw = qld.FrameWindow(8, 8, 2, bits=12)
    with pytest.raises(ValueError):
        fw.update(torch.zeros((8, 9), dtype=torch.int16, device="cuda"))
    assert qld.FrameWindow.bytes(8, 8, 2, bits=12) == 4 * 2 * 64 * 2 + 64 * 8
    fw.close()
