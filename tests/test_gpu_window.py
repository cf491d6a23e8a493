"""GPU parity of the sliding window and of the serving loop against the oracle's
brute-force window (which re-sums the stored history and never subtracts).

Bar: I/Q bit-exact after every cycle, amplitude within 2 ulp; each stream's
results in a mixed, continuously batched run identical to the same stream
run alone.
"""
import os
import tempfile
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1511_03390_amd as qld
import scenes
from tests.gpu_util import amp_ulps, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W,M,bits,dt,n", [(9, 13, 5, 12, np.uint16, 13), (32, 64, 16, 16, np.uint16, 40),
                                             (7, 40, 3, 8, np.uint8, 10), (1, 1, 1, 12, np.uint16, 4)])
def test_window_matches_brute_force_every_cycle(H, W, M, bits, dt, n):
    need_gpu()
    rng = np.random.default_rng(H * W + M)
    say("window", H, W, M, bits, n)
    cycles = [rng.integers(0, 1 << bits, size=(4, H, W)).astype(dt) for _ in range(n)]
    win = qld.Window(H, W, M, dtype=torch.uint8 if dt == np.uint8 else torch.int16, bits=bits)
    I = torch.empty((H, W), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    amp = torch.empty((H, W), dtype=torch.float32, device="cuda")
    for c, (oI, oQ, nin) in enumerate(oracle.window_series(cycles, M)):
        warm = win.update(to_dev(cycles[c]), I, Q, amp)
        torch.cuda.synchronize()
        assert warm == (1 if c + 1 >= M else 0)
        assert np.array_equal(I.cpu().numpy(), oI) and np.array_equal(Q.cpu().numpy(), oQ), c
        assert amp_ulps(amp.cpu().numpy(), oracle.amplitude(oI, oQ)).max() <= 2.0
    assert win.info() == (min(n, M), n)
    win.close()


def test_window_reset_and_checkpoint_resume():
    need_gpu()
    H, W, M = 12, 20, 6
    rng = np.random.default_rng(5)
    cycles = [rng.integers(0, 4096, size=(4, H, W)).astype(np.uint16) for _ in range(20)]
    ref = list(oracle.window_series(cycles, M, resets=[8]))
    win = qld.Window(H, W, M, bits=12)
    I = torch.empty((H, W), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "w.ckpt")
        for c in range(20):
            if c == 8:
                win.reset()
            if c == 14:
                win.save(path)
                win.close()
                win = qld.Window(H, W, M, bits=12)
                win.load(path)
            win.update(to_dev(cycles[c]), I, Q)
            torch.cuda.synchronize()
            assert np.array_equal(I.cpu().numpy(), ref[c][0]) and np.array_equal(Q.cpu().numpy(), ref[c][1]), c
        other = qld.Window(H, W + 1, M, bits=12)
        with pytest.raises(qld.QldError) as e:
            other.load(path)
        assert e.value.status == qld.E_STATE
    win.close()


def test_window_sinusoid_closed_form():
    need_gpu()
    a, b, c0 = 3, -4, 50
    cyc = np.broadcast_to(np.array([c0 + a, c0 + b, c0 - a, c0 - b], dtype=np.uint16)[:, None, None],
                          (4, 3, 16)).copy()
    win = qld.Window(3, 16, 7, bits=12)
    I = torch.empty((3, 16), dtype=torch.int32, device="cuda")
    Q = torch.empty_like(I)
    amp = torch.empty((3, 16), dtype=torch.float32, device="cuda")
    for k in range(12):
        win.update(to_dev(cyc), I, Q, amp)
        torch.cuda.synchronize()
        n = min(k + 1, 7)
        assert (I.cpu().numpy() == 2 * n * a).all() and (Q.cpu().numpy() == 2 * n * b).all()
        assert (amp.cpu().numpy() == 2 * n * 5).all()


# ---------------------------------------------------------------------------
# Serving: alone vs in the mix, admission by budget, gaps.
# ---------------------------------------------------------------------------

def run_server(streams, n_cycles, M, budget=None, interleave=True, Ms=0, held=False, whole_cycles=False):
    """Submit ``n_cycles`` cycles of each (H, W, seed) stream; return per-stream
    {cycle: (I, Q, amp[, Is, Qs])} read back right after each poll.
    held: the scheduler is drained and held while each round of cycles (one
    per stream) is submitted, and released after it, so each round is one
    launch carrying every stream.
    whole_cycles: cycles go in with qld_stream_submit_cycle instead of four
    single-frame submits."""
    need = 0
    srv = qld.Server(budget or (1 << 34), out_slots=64, keep_iq=True)
    ids = []
    cams = []
    for (H, W, seed) in streams:
        sid, ok = srv.open(H, W, M, M_short=Ms, bits=16)
        assert ok
        ids.append(sid)
        cams.append(scenes.CameraStream(H, W, seed, bits=16, bank=4))
    out = {sid: {} for sid in ids}

    def collect():
        for r in srv.poll():
            H, W = r.H, r.W
            amp = qld.device_view(r.amp, (H, W), torch.float32).cpu().numpy().copy()
            pI, pQ, pIs, pQs = srv.result_iq(r)
            I = qld.device_view(pI, (H, W), torch.int32).cpu().numpy().copy()
            Q = qld.device_view(pQ, (H, W), torch.int32).cpu().numpy().copy()
            extra = ()
            if Ms:
                extra = (qld.device_view(pIs, (H, W), torch.int32).cpu().numpy().copy(),
                         qld.device_view(pQs, (H, W), torch.int32).cpu().numpy().copy())
            out[r.stream_id][r.cycle] = (I, Q, amp) + extra

    frames = [[cam.cycle(c) for c in range(n_cycles)] for cam in cams]
    order = [(c, j, s) for c in range(n_cycles) for j in range(4) for s in range(len(ids))] if interleave else \
        [(c, j, s) for s in range(len(ids)) for c in range(n_cycles) for j in range(4)]
    if whole_cycles:
        order = [o for o in order if o[1] == 0]
    for (c, j, s) in order:
        if held and s == 0 and j == 0:
            srv.drain()          # the previous round is done: its staging slots are free
            srv.hold(True)
        if whole_cycles:
            st = srv.submit_cycle(ids[s], np.ascontiguousarray(frames[s][c]), 4 * c, time.monotonic_ns())
        else:
            st = srv.submit(ids[s], frames[s][c][j], 4 * c + j, time.monotonic_ns())
        assert st == qld.OK, (c, j, s, st)
        if held and s == len(ids) - 1 and (j == 3 or whole_cycles):
            srv.hold(False)
        if (j == 3 or whole_cycles) and c % 8 == 7:
            collect()
    srv.drain()
    collect()
    st = srv.stats()
    srv.close()
    return [out[sid] for sid in ids], frames, st


def test_server_alone_vs_mix_and_oracle():
    """Three streams of different sizes, each cycle of the three staged while
    the scheduler is held and launched together: every launch is a mix of all
    three (the batched kernel's job lookup for jobs 1 and 2 runs).  Each
    stream's I/Q/amplitude after every cycle equals the same stream run alone
    (unheld, one launch per cycle) and the oracle's re-summing window."""
    need_gpu()
    shapes = [(48, 80, 11), (96, 64, 12), (40, 136, 13)]
    M, n = 6, 16
    mixed, frames, st = run_server(shapes, n, M, held=True)
    say("server stats", st)
    assert st["cycles"] == 3 * n
    assert st["max_streams_in_batch"] == 3
    assert st["batches"] == n
    for k, shp in enumerate(shapes):
        alone, _, sta = run_server([shp], n, M)
        assert sta["max_streams_in_batch"] == 1
        for c in range(n):
            for a, b in zip(alone[0][c], mixed[k][c]):
                assert np.array_equal(a, b), (shp, c)
        ref = list(oracle.window_series(frames[k], M))
        for c in range(n):
            I, Q, amp = mixed[k][c]
            assert np.array_equal(I, ref[c][0]) and np.array_equal(Q, ref[c][1]), (shp, c)
            assert amp_ulps(amp, oracle.amplitude(ref[c][0], ref[c][1])).max() <= 2.0


def test_server_full_size_three_cameras_sampled():
    """The benchmark's streaming configuration at full size: 640x512,
    1280x1024 and 2048x2048 uint16 cameras in one server (M = 64, 16 output
    slots), 8 distinct cycles per camera replayed, 70 cycles so the ring wraps.
    64 sampled pixels per stream checked against the oracle's re-summing window
    at cycles 0, 31, 63, 64 and 69."""
    need_gpu()
    M, n, bank = 64, 70, 8
    check = {0, 31, 63, 64, 69}
    srv = qld.Server(1 << 36, out_slots=16, keep_iq=True)
    rng = np.random.default_rng(303)
    ids, banks, picks = [], [], []
    for k, (h, w) in enumerate(scenes.STREAM_SHAPES):
        sid, ok = srv.open(h, w, M, bits=16)
        assert ok
        ids.append(sid)
        cam = scenes.CameraStream(h, w, scenes.seed_for(3, k), bits=16, bank=8)
        banks.append([cam.cycle(c) for c in range(bank)])
        picks.append((rng.integers(0, h, 64), rng.integers(0, w, 64)))
    say("full-size streams", scenes.STREAM_SHAPES)
    got = {sid: {} for sid in ids}

    def collect():
        for r in srv.poll():
            if r.cycle not in check:
                continue
            k = ids.index(r.stream_id)
            ys, xs = picks[k]
            pI, pQ, _, _ = srv.result_iq(r)
            I = qld.device_view(pI, (r.H, r.W), torch.int32).cpu().numpy()[ys, xs]
            Q = qld.device_view(pQ, (r.H, r.W), torch.int32).cpu().numpy()[ys, xs]
            amp = qld.device_view(r.amp, (r.H, r.W), torch.float32).cpu().numpy()[ys, xs]
            got[r.stream_id][r.cycle] = (I, Q, amp)

    for c in range(n):
        for j in range(4):
            for k, sid in enumerate(ids):
                assert srv.submit(sid, banks[k][c % bank][j], 4 * c + j, time.monotonic_ns()) == qld.OK
        if c % 4 == 3:
            srv.drain()
            collect()
    srv.drain()
    collect()
    srv.close()
    for k, sid in enumerate(ids):
        ys, xs = picks[k]
        series = [np.ascontiguousarray(np.asarray(banks[k][c % bank])[:, ys, xs][:, None, :]) for c in range(n)]  # [4][1][64]
        ref = list(oracle.window_series(series, M))
        for c in sorted(check):
            I, Q, amp = got[sid][c]
            assert np.array_equal(I, ref[c][0][0]) and np.array_equal(Q, ref[c][1][0]), (k, c)
            assert amp_ulps(amp, oracle.amplitude(ref[c][0][0], ref[c][1][0])).max() <= 2.0, (k, c)


def test_server_whole_cycle_submit_and_result_validity():
    """qld_stream_submit_cycle (one host copy and one transfer per cycle) gives
    the same images as frame-by-frame submits; while held, a fifth staged
    cycle is refused with QLD_E_AGAIN and taken after the release; a result
    stays valid until its output slot is relaunched."""
    need_gpu()
    shapes = [(40, 72, 31), (17, 200, 32)]
    M, n = 5, 12
    by_cycle, frames, st = run_server(shapes, n, M, whole_cycles=True, held=True)
    assert st["max_streams_in_batch"] == 2 and st["cycles"] == 2 * n and st["batches"] == n
    by_frame, _, _ = run_server(shapes, n, M)
    for k in range(len(shapes)):
        ref = list(oracle.window_series(frames[k], M))
        for c in range(n):
            for a, b in zip(by_cycle[k][c], by_frame[k][c]):
                assert np.array_equal(a, b), (k, c)
            assert np.array_equal(by_cycle[k][c][0], ref[c][0]) and np.array_equal(by_cycle[k][c][1], ref[c][1])

    H, W = 24, 40
    srv = qld.Server(1 << 32, out_slots=2, keep_iq=True)
    sid, ok = srv.open(H, W, 3, bits=16)
    assert ok
    cam = scenes.CameraStream(H, W, 33, bits=16, bank=8)
    cyc = [np.ascontiguousarray(cam.cycle(c)) for c in range(8)]
    srv.hold(True)
    for c in range(4):
        assert srv.submit_cycle(sid, cyc[c], 4 * c, 0) == qld.OK
    assert srv.submit_cycle(sid, cyc[4], 16, 0) == qld.E_AGAIN       # staging full, nothing launched
    assert srv.submit(sid, cyc[4][0], 16, 0) == qld.E_AGAIN
    assert srv.poll() == []
    srv.hold(False)
    srv.drain()
    first = srv.poll()
    assert [r.cycle for r in first] == [0, 1, 2, 3] and [r.seq for r in first] == [0, 1, 2, 3]
    # Two output slots: cycles 0 and 1 were overwritten by 2 and 3.
    assert [srv.result_valid(r) for r in first] == [False, False, True, True]
    assert srv.submit_cycle(sid, cyc[4], 16, 0) == qld.OK
    assert srv.submit_cycle(sid, cyc[6], 24, 0) == qld.E_GAP           # cycle 5 missing: new window
    with pytest.raises(qld.QldError):
        srv.submit_cycle(sid, cyc[7], 26, 0)                           # not a cycle start
    srv.drain()
    rest = srv.poll()
    assert [r.cycle for r in rest] == [4, 6]
    assert not srv.result_valid(first[2]) and srv.result_valid(rest[1])
    pI, pQ, _, _ = srv.result_iq(rest[1])
    I = qld.device_view(pI, (H, W), torch.int32).cpu().numpy()
    assert np.array_equal(I, oracle.qld(cyc[6])[0])
    ref = list(oracle.window_series(cyc[:5], 3))
    pI, pQ, _, _ = srv.result_iq(rest[0])
    assert np.array_equal(qld.device_view(pI, (H, W), torch.int32).cpu().numpy(), ref[4][0])
    srv.close()


def test_server_submit_from_page_locked_frames():
    """Frames in page-locked host memory are copied straight from the
    caller's buffer (one copy fewer); the call waits for that copy, so the
    buffer can be refilled at once.  One reused page-locked buffer, per cycle
    and per frame, gives the oracle's window every cycle."""
    need_gpu()
    H, W, M, n = 33, 104, 4, 10
    srv = qld.Server(1 << 32, out_slots=16, keep_iq=True)
    sid, ok = srv.open(H, W, M, bits=16)
    assert ok
    cam = scenes.CameraStream(H, W, 77, bits=16, bank=8)
    cyc = [np.ascontiguousarray(cam.cycle(c)) for c in range(n)]
    pin = torch.empty((4, H, W), dtype=torch.int16, pin_memory=True)
    pv = pin.numpy().view(np.uint16)
    got = {}

    def collect():
        for r in srv.poll():
            pI, pQ, _, _ = srv.result_iq(r)
            got[r.cycle] = (qld.device_view(pI, (H, W), torch.int32).cpu().numpy(),
                            qld.device_view(pQ, (H, W), torch.int32).cpu().numpy())

    for c in range(n):
        if c % 2 == 0:
            pv[...] = cyc[c]
            assert srv.submit_cycle(sid, pv, 4 * c, 0) == qld.OK
        else:
            for j in range(4):
                pv[0] = cyc[c][j]
                assert srv.submit(sid, pv[0], 4 * c + j, 0) == qld.OK
        srv.drain()
        collect()
    ref = list(oracle.window_series(cyc, M))
    for c in range(n):
        assert np.array_equal(got[c][0], ref[c][0]) and np.array_equal(got[c][1], ref[c][1]), c
    srv.close()


def test_server_short_window_shares_ring():
    need_gpu()
    M, Ms, n = 8, 3, 14
    res, frames, _ = run_server([(24, 40, 21)], n, M, Ms=Ms)
    longw = list(oracle.window_series(frames[0], M))
    shortw = list(oracle.window_series(frames[0], Ms))
    for c in range(n):
        I, Q, amp, Is, Qs = res[0][c]
        assert np.array_equal(I, longw[c][0]) and np.array_equal(Is, shortw[c][0])
        assert np.array_equal(Q, longw[c][1]) and np.array_equal(Qs, shortw[c][1])


def test_server_admission_by_budget_and_gap_reset():
    need_gpu()
    srv = qld.Server(1 << 40, out_slots=4, keep_iq=True)
    b_small = srv.stream_bytes(64, 64, 8, bits=16)
    b_big = srv.stream_bytes(128, 128, 8, bits=16)
    srv.close()
    srv = qld.Server(b_big + b_small, out_slots=4, keep_iq=True)
    s1, ok1 = srv.open(128, 128, 8, bits=16)
    s2, ok2 = srv.open(64, 64, 8, bits=16)
    s3, ok3 = srv.open(64, 64, 8, bits=16)
    assert ok1 and ok2 and not ok3
    assert srv.state(s3) == qld.STREAM_PENDING
    cam = scenes.CameraStream(64, 64, 5, bits=16, bank=4)
    assert srv.submit(s3, cam.cycle(0)[0], 0, 0) == qld.E_AGAIN
    with pytest.raises(qld.QldError) as e:
        qld.Server(1 << 20).open(4096, 4096, 64, bits=16)
    assert e.value.status == qld.E_BUDGET
    srv.close_stream(s1)
    assert srv.state(s3) == qld.STREAM_ACTIVE
    # Gap: frames 0..5 then 9.. -> the window restarts at cycle 3 (frame 12).
    frames = [cam.cycle(c) for c in range(6)]
    for f in range(6):
        srv.submit(s3, frames[f // 4][f % 4], f, 0)
    assert srv.submit(s3, frames[2][1], 9, 0) == qld.E_GAP
    for f in range(10, 24):
        srv.submit(s3, frames[f // 4][f % 4], f, 0)
    srv.drain()
    got = {}
    for r in srv.poll():
        pI, pQ, _, _ = srv.result_iq(r)
        got[r.cycle] = qld.device_view(pI, (64, 64), torch.int32).cpu().numpy().copy()
    assert sorted(got) == [0, 3, 4, 5]
    ref = list(oracle.window_series([frames[3], frames[4], frames[5]], 8))
    for k, c in enumerate((3, 4, 5)):
        assert np.array_equal(got[c], ref[k][0])
    assert np.array_equal(got[0], oracle.qld(frames[0])[0])
    srv.close()
