"""GPU tests of a LEARNED serving stream: short window M_S and long window M
on one ring, the denoiser run on every cycle's short-window I/Q, the gate's
choice between its image and the plain long-window amplitude per cycle.

Bars: the plain amplitude within 2 ulp and the short-window I/Q bit-exact
against the oracle's brute-force windows (resets included); the served image,
gate and flag bit-exact against the same library entry points called one by
one on the same inputs (qld_denoise_prepare with the exact host sample sums,
qld_denoiser_forward), whose own parity against the oracle is tested in
test_gpu_learned.py; a PLAIN stream in the same launches unchanged.
"""
import math
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1511_03390_amd as qld
import scenes
from paper_1511_03390_amd import learned as Lr
from tests.gpu_util import amp_ulps, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def poisson_cycles(rng, n, H, W, lam=2000.0):
    return [np.minimum(rng.poisson(lam, size=(4, H, W)), 4095).astype(np.uint16) for _ in range(n)]


def view(ptr, H, W, dt):
    return qld.device_view(ptr, (H, W), dt).cpu().numpy().copy()


def run(H, W, M, Ms, cycles, thr, gap_after=None, out_slots=32, seed=3, with_plain=None, drain_each=False):
    srv = qld.Server(1 << 34, out_slots=out_slots)
    sid, ok = srv.open(H, W, M, M_short=Ms, bits=12, mode=qld.MODE_LEARNED)
    assert ok
    with pytest.raises(qld.QldError) as e:
        srv.submit(sid, cycles[0][0], 0, time.monotonic_ns())
    assert e.value.status == qld.E_STATE
    dn = qld.Denoiser(H, W, 1)
    dn.set_params(Lr.he_init(seed))
    srv.set_denoiser(sid, dn, thr)
    pid = None
    if with_plain:
        pid, ok = srv.open(*with_plain[0], M, bits=12)
        assert ok
    out, pout = {}, {}

    def collect():
        for r in srv.poll(1024):
            if r.stream_id == sid:
                _, _, pIs, pQs = srv.result_iq(r)
                out[r.cycle] = dict(served=view(r.amp, H, W, torch.float32),
                                    plain=view(r.amp_plain, H, W, torch.float32),
                                    Is=view(pIs, H, W, torch.int32), Qs=view(pQs, H, W, torch.int32),
                                    gate=float(r.gate), learned=int(r.learned), warm=int(r.warm))
            else:
                pout[r.cycle] = view(r.amp, r.H, r.W, torch.float32)

    f = 0
    for c, cyc in enumerate(cycles):
        for j in range(4):
            srv.submit(sid, cyc[j], f + j, time.monotonic_ns())
            if pid is not None:
                srv.submit(pid, with_plain[1][c][j], 4 * c + j, time.monotonic_ns())
        f += 4
        if gap_after is not None and c == gap_after:
            f += 4                                     # one cycle lost: the window restarts
        if drain_each:
            srv.drain()
            collect()
    srv.drain()
    collect()
    srv.close()
    return out, pout, dn


def window_sums(cycles, c, Ms):
    """Each pixel's and the frame's sample sums over window cycles c - Ms + 1 .. c."""
    P = sum(cycles[j].astype(np.int64).sum(axis=0) for j in range(c - Ms + 1, c + 1))
    return P, int(P.sum())


def reproduce(dn, Is, Qs, psum_S, sum_S, Ms):
    """The served image of one cycle from the library's entry points, called one by one."""
    H, W = Is.shape
    I_d = torch.from_numpy(Is[None]).cuda()
    Q_d = torch.from_numpy(Qs[None]).cuda()
    p_d = torch.from_numpy(psum_S.astype(np.uint32).view(np.int32)[None]).cuda()
    s_d = torch.tensor([sum_S], dtype=torch.int64).cuda()
    x, scale = qld.denoise_prepare(I_d, Q_d, p_d, s_d, Ms)
    y = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    g = torch.empty(1, dtype=torch.float32, device="cuda")
    dn.forward(x, y, g)
    torch.cuda.synchronize()
    return (y[0] * scale[0]).cpu().numpy(), float(g.item())


def check(out, cycles, M, Ms, thr, resets=(), dn=None):
    longw = list(oracle.window_series(cycles, M, resets=list(resets)))
    shortw = list(oracle.window_series(cycles, Ms, resets=list(resets)))
    starts = [0] + list(resets)
    n_learned = 0
    for k in range(len(cycles)):
        cam = k + (1 if resets and k >= resets[0] else 0)
        r = out[cam]
        c = k - max(s for s in starts if s <= k)           # window cycle index
        assert np.array_equal(r["Is"], shortw[k][0]) and np.array_equal(r["Qs"], shortw[k][1]), k
        assert amp_ulps(r["plain"], oracle.amplitude(longw[k][0], longw[k][1])).max() <= 2.0, k
        inv_n = np.float32(1.0) / np.float32(min(c + 1, M))
        plain_pc = r["plain"].astype(np.float32) * inv_n
        if c + 1 >= Ms:
            P, sum_S = window_sums(cycles, k, Ms)
            y, g = reproduce(dn, r["Is"], r["Qs"], P, sum_S, Ms)
            assert r["gate"] == g, (k, r["gate"], g)
            use = g <= thr
            assert r["learned"] == int(use), k
            assert np.array_equal(r["served"], y if use else plain_pc), k
            n_learned += int(use)
        else:
            assert math.isnan(r["gate"]) and r["learned"] == 0, k
            assert np.array_equal(r["served"], plain_pc), k
        assert r["warm"] == (1 if c + 1 >= M else 0)
    return n_learned


@pytest.mark.parametrize("H,W,M,Ms,n,drain_each", [(40, 72, 8, 3, 20, False), (17, 130, 5, 5, 9, True),
                                                   (64, 64, 12, 1, 14, False)])
def test_learned_stream_serves_denoiser_output(H, W, M, Ms, n, drain_each):
    need_gpu()
    say("learned stream", H, W, M, Ms, n, drain_each)
    rng = np.random.default_rng(H * W + Ms)
    cycles = poisson_cycles(rng, n, H, W)
    out, _, dn = run(H, W, M, Ms, cycles, float("inf"), drain_each=drain_each)
    assert sorted(out) == list(range(n))
    nl = check(out, cycles, M, Ms, float("inf"), dn=dn)
    assert nl == n - (Ms - 1)
    dn.close()


def test_learned_stream_full_size_sampled():
    """The clutter-and-motion serving configuration's shape: one LEARNED
    1024 x 1024 stream, M_S = 16 and M = 128 on one ring, 132 cycles (a bank of
    8 Poisson cycles replayed) so the long window wraps.  At cycles 15, 127
    and 131: short-window I/Q bit-exact and the plain amplitude within 2 ulp on
    64 sampled pixels against the oracle's windows; the served image and gate
    bit-exact against the entry points called one by one on the full image."""
    need_gpu()
    H = W = 1024
    M, Ms, n, nb = 128, 16, 132, 8
    check_at = {15, 127, 131}
    rng = np.random.default_rng(1511033905)
    bank = poisson_cycles(rng, nb, H, W)
    srv = qld.Server(1 << 36, out_slots=16)
    sid, ok = srv.open(H, W, M, M_short=Ms, bits=12, mode=qld.MODE_LEARNED)
    assert ok
    dn = qld.Denoiser(H, W, 1)
    dn.set_params(Lr.he_init(5))
    srv.set_denoiser(sid, dn, float("inf"))
    got = {}

    def collect():
        for r in srv.poll(256):
            if r.cycle in check_at:
                _, _, pIs, pQs = srv.result_iq(r)
                got[r.cycle] = dict(served=view(r.amp, H, W, torch.float32),
                                    plain=view(r.amp_plain, H, W, torch.float32),
                                    Is=view(pIs, H, W, torch.int32), Qs=view(pQs, H, W, torch.int32),
                                    gate=float(r.gate), learned=int(r.learned), warm=int(r.warm))

    say("learned stream full size", H, W, M, Ms, n)
    for c in range(n):
        for j in range(4):
            assert srv.submit(sid, bank[c % nb][j], 4 * c + j, time.monotonic_ns()) == qld.OK
        if c % 4 == 3:
            srv.drain()
            collect()
    srv.drain()
    collect()
    srv.close()
    assert sorted(got) == sorted(check_at)
    ys, xs = rng.integers(0, H, 64), rng.integers(0, W, 64)
    series = [np.ascontiguousarray(bank[c % nb][:, ys, xs][:, None, :]) for c in range(n)]
    longw = list(oracle.window_series(series, M))
    shortw = list(oracle.window_series(series, Ms))
    for c in sorted(check_at):
        r = got[c]
        assert np.array_equal(r["Is"][ys, xs], shortw[c][0][0]) and np.array_equal(r["Qs"][ys, xs], shortw[c][1][0]), c
        assert amp_ulps(r["plain"][ys, xs], oracle.amplitude(longw[c][0][0], longw[c][1][0])).max() <= 2.0, c
        P, sum_S = window_sums([bank[j % nb] for j in range(c + 1)], c, Ms)
        y, g = reproduce(dn, r["Is"], r["Qs"], P, sum_S, Ms)
        assert r["gate"] == g and r["learned"] == 1, c
        assert np.array_equal(r["served"], y), c
        assert r["warm"] == (1 if c + 1 >= M else 0), c
    dn.close()


def test_learned_stream_gate_fallback_reset_and_plain_neighbour():
    need_gpu()
    H, W, M, Ms, n = 32, 48, 6, 2, 16
    rng = np.random.default_rng(77)
    cycles = poisson_cycles(rng, n, H, W)
    ph, pw = 24, 40
    pcyc = poisson_cycles(rng, n, ph, pw)
    # Every cycle falls back (threshold below any gate), the stream loses one
    # cycle after cycle 6, and a PLAIN stream shares the launches.
    out, pout, dn = run(H, W, M, Ms, cycles, float("-inf"), gap_after=6, with_plain=((ph, pw), pcyc))
    nl = check(out, cycles, M, Ms, float("-inf"), resets=(7,), dn=dn)
    assert nl == 0
    ref = list(oracle.window_series(pcyc, M))
    for c in range(n):
        assert amp_ulps(pout[c], oracle.amplitude(ref[c][0], ref[c][1])).max() <= 2.0, c
    # A threshold between the gates: the flag follows the gate cycle by cycle.
    gates = sorted(v["gate"] for v in out.values() if not math.isnan(v["gate"]))
    thr = gates[len(gates) // 2]
    out2, _, dn2 = run(H, W, M, Ms, cycles, thr, gap_after=6)
    nl2 = check(out2, cycles, M, Ms, thr, resets=(7,), dn=dn2)
    say("gate threshold", thr, "learned cycles", nl2, "of", len(gates))
    assert 0 < nl2 <= len(gates)
    dn.close()
    dn2.close()


def test_learned_stream_arguments():
    need_gpu()
    srv = qld.Server(1 << 30, out_slots=4)
    with pytest.raises(qld.QldError) as e:          # LEARNED needs a short window
        srv.open(16, 16, 8, M_short=0, bits=12, mode=qld.MODE_LEARNED)
    assert e.value.status == qld.E_INVAL
    sid, _ = srv.open(16, 16, 8, M_short=2, bits=12, mode=qld.MODE_LEARNED)
    pid, _ = srv.open(16, 16, 8, bits=12)
    dn = qld.Denoiser(16, 24, 1)
    with pytest.raises(qld.QldError) as e:
        srv.set_denoiser(sid, dn)
    assert e.value.status == qld.E_SHAPE
    dn2 = qld.Denoiser(16, 16, 1)
    with pytest.raises(qld.QldError) as e:
        srv.set_denoiser(pid, dn2)
    assert e.value.status == qld.E_STATE
    assert srv.stream_bytes(16, 16, 8, 2, bits=12, mode=qld.MODE_LEARNED) > srv.stream_bytes(16, 16, 8, 2, bits=12)
    srv.close()
    dn.close()
    dn2.close()
