"""The entry point that allocates nothing (qld_lockin_image_noalloc), through the
C ABI, against qld_lockin_image on the same inputs: I/Q, amplitude and the
frame statistics bit-identical, call after call on the shared scratch array
(each later call smaller than the one before), and a call needing more scratch
than the array holds refused before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1511_03390_amd as qld
import scenes
from tests.gpu_util import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def outputs(H, W, T):
    dev = torch.device("cuda")
    return (torch.full((H, W), 7, dtype=torch.int32, device=dev), torch.full((H, W), -7, dtype=torch.int32, device=dev),
            torch.full((H, W), -1.0, dtype=torch.float32, device=dev),
            torch.full((T,), 123, dtype=torch.int64, device=dev), torch.full((T,), 45, dtype=torch.int32, device=dev))


def both(frames, bits, phase0, stats=True):
    """(qld_lockin_image, qld_lockin_image_noalloc) results on one stack, as host arrays."""
    T, H, W = frames.shape
    res = []
    for f in (qld.lockin_image, qld.lockin_image_noalloc):
        I, Q, amp, fs, fc = outputs(H, W, T)
        f(frames, I, Q, amp, phase0=phase0, bits=bits, frame_sum=fs if stats else None,
          frame_sat=fc if stats else None)
        torch.cuda.synchronize()
        res.append([x.cpu().numpy() for x in (I, Q, amp, fs, fc)])
    return res


# Calls in this order share the scratch array; each is smaller than the one
# before.  (dtype, T, H, W, phase0, bits): a split tail past one round of
# wide tiles (1050 tiles of 4096 8-bit pixels, 525 wide tiles of 2 on 512
# work-groups: statistics and I/Q partials), a small image split over the
# frames (I/Q partials from many splits), and a ragged image with a scalar
# column tail (both kernels' statistics rows).
SEQUENCE = [
    (np.uint8, 130, 2100, 2048, 1, 8),
    (np.uint16, 1029, 40, 64, 3, 12),
    (np.uint16, 67, 300, 257, 2, 12),
]


def test_noalloc_matches_lockin_image_call_after_call():
    need_gpu()
    for k, (dt, T, H, W, phase0, bits) in enumerate(SEQUENCE):
        say("noalloc call", k, dt.__name__, T, H, W, phase0, bits)
        rng = np.random.default_rng(77 + k)
        buf, _ = scenes.random_stack(rng, T, H, W, dt, bits=bits)
        top = (1 << bits) - 1
        buf[rng.random(buf.shape) < 1e-4] = top
        frames = to_dev(buf)
        (a, b) = both(frames, bits, phase0)
        for name, x, y in zip(("I", "Q", "amp", "frame_sum", "frame_sat"), a, b):
            assert np.array_equal(x, y), "%s differs from qld_lockin_image (call %d)" % (name, k)
        if H * W * T <= 10 ** 7:       # small enough for the oracle to confirm as well
            oI, oQ = oracle.qld(buf, phase0)
            assert np.array_equal(b[0].astype(np.int64), oI) and np.array_equal(b[1].astype(np.int64), oQ)
            s, n = oracle.frame_stats(buf, bits)
            assert np.array_equal(b[3].astype(np.uint64), s) and np.array_equal(b[4].astype(np.uint32), n)


def test_noalloc_refuses_more_scratch_than_it_holds():
    need_gpu()
    # An unaligned 8-bit stack takes the one-pixel-per-lane kernel: four
    # statistics rows of 8 bytes per frame for every 256 pixels.
    H, W, T = 1024, 1024, 257
    need = (H * W // 256) * 4 * 8 * T
    assert need > qld.NOALLOC_SCRATCH_BYTES
    raw = torch.zeros(T * H * W + 16, dtype=torch.uint8, device="cuda")
    frames = raw[1:1 + T * H * W].view(T, H, W)
    I, Q, amp, fs, fc = outputs(H, W, T)
    d = qld.frame_desc(frames, 8)
    st = qld.lib.qld_lockin_image_noalloc(qld._ptr(frames), ctypes.byref(d), T, 0, qld._ptr(I), qld._ptr(Q),
                                          qld._ptr(amp), qld._ptr(fs), qld._ptr(fc), qld._stream(None))
    assert st == qld.E_NOMEM
    assert b"scratch" in qld.lib.qld_last_error()
    torch.cuda.synchronize()
    assert int((I != 7).sum()) == 0 and int((fs != 123).sum()) == 0, "a refused call wrote its outputs"
    # Without statistics the same stack needs no scratch and runs.
    raw[1:1 + T * H * W].view(T, H, W)[::3] = 5
    (a, b) = both(frames, 8, 0, stats=False)
    for name, x, y in zip(("I", "Q", "amp"), a[:3], b[:3]):
        assert np.array_equal(x, y), name
