"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms
of the lock-in sums (sinusoids, DC, ramps, clutter, drift), a textbook FFT,
exact integer identities (impulse basis, linearity, cycle permutation, phase
rotation, frame splitting), the overflow edge, and the paper's worked CNR
geometry.  A dropped term, a wrong sign or index, or swapped quadratures
fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import judges
from tests.golden.fixtures import read_kv


def stack_from_series(series, H=1, W=1, dtype=np.uint16):
    s = np.asarray(series, dtype=np.int64)
    assert s.min() >= 0 and s.max() <= np.iinfo(dtype).max
    return np.broadcast_to(s[:, None, None], (len(s), H, W)).astype(dtype).copy()


def test_reference_tables_are_exact_integers():
    c, s = oracle.reference_tables()
    assert c == [1, 0, -1, 0] and s == [0, 1, 0, -1]


@pytest.mark.parametrize("phase0", [0, 1, 2, 3, 7, -1])
def test_impulse_basis(phase0):
    # A unit sample in frame t contributes (cos, sin) of phase (phase0 + t) * pi / 2.
    T = 8
    for t in range(T):
        series = np.zeros(T, dtype=np.int64)
        series[t] = 1
        I, Q = oracle.qld(stack_from_series(series), phase0)
        th = math.pi * (phase0 + t) / 2.0
        assert I[0, 0] == round(math.cos(th)) and Q[0, 0] == round(math.sin(th))


@pytest.mark.parametrize("a,b", [(3, 4), (4, -3), (-3, -4), (5, 0), (0, 5), (0, -5)])
def test_sinusoid_amplitude_is_phase_independent(a, b):
    # x_t = c + a cos(pi t/2) + b sin(pi t/2) = c + A cos(pi t/2 - psi), A = 5:
    # I = 2 M a, Q = 2 M b, R = 2 M A for every phase psi.
    M, c = 16, 1000
    t = np.arange(4 * M)
    x = c + a * np.rint(np.cos(np.pi * t / 2)).astype(int) + b * np.rint(np.sin(np.pi * t / 2)).astype(int)
    I, Q = oracle.qld(stack_from_series(x, 2, 3))
    assert (I == 2 * M * a).all() and (Q == 2 * M * b).all()
    R = oracle.amplitude(I, Q)
    assert (R == 2 * M * 5).all()


def test_dc_cancels_exactly():
    for c in (0, 1, 255, 4095, 65535):
        I, Q = oracle.qld(stack_from_series([c] * 64, 3, 5))
        assert not I.any() and not Q.any()


@pytest.mark.parametrize("phi", [0.3, 1.1, 2.0, 4.0, 5.9])
def test_square_wave_amplitude(phi):
    # +A where cos(pi t/2 + phi) >= 0, -A elsewhere; off sample boundaries
    # |I| = |Q| = 2 M A, so R = 2 sqrt(2) M A.
    M, A, c = 16, 4, 100
    t = np.arange(4 * M)
    sq = np.where(np.cos(np.pi * t / 2 + phi) >= 0, A, -A)
    I, Q = oracle.qld(stack_from_series(c + sq, dtype=np.uint8))
    assert abs(I[0, 0]) == 2 * M * A and abs(Q[0, 0]) == 2 * M * A
    assert abs(oracle.amplitude(I, Q)[0, 0] - 2 * math.sqrt(2) * M * A) < 1e-9


def test_linear_ramp_leaves_bias():
    # x_t = a + b t: I = Q = -2 b M (linear drift does not cancel).
    M, a, b = 10, 500, 3
    I, Q = oracle.qld(stack_from_series(a + b * np.arange(4 * M)))
    assert I[0, 0] == -2 * b * M and Q[0, 0] == -2 * b * M


@pytest.mark.parametrize("M", [6, 7])
def test_clutter_at_one_and_a_half_fmod(M):
    # x_t = c + rint(A cos(3 pi t/4 + psi)) flips sign every cycle, so whole
    # pairs of cycles cancel; an odd count leaves exactly one cycle.
    A, c, psi = 700, 2000, 0.37
    t = np.arange(4 * M)
    x = c + np.rint(A * np.cos(3 * np.pi * t / 4 + psi)).astype(np.int64)
    I, Q = oracle.qld(stack_from_series(x))
    if M % 2 == 0:
        assert I[0, 0] == 0 and Q[0, 0] == 0
    else:
        I1, Q1 = oracle.qld(stack_from_series(x[:4]))
        assert I[0, 0] == I1[0, 0] and Q[0, 0] == Q1[0, 0] and (I1[0, 0], Q1[0, 0]) != (0, 0)


def test_phase_drift_attenuation():
    # Phase drifting delta rad/cycle: R = 2 M A |sin(M delta/2) / (M sin(delta/2))|,
    # up to the rounding of the samples (each off by <= 0.5, so |dI|, |dQ| <= 0.5*2M).
    M, A, c, delta, phi0 = 128, 20000.0, 30000, 0.01, 0.4
    t = np.arange(4 * M)
    x = c + np.rint(A * np.cos(np.pi * t / 2 + phi0 + delta * (t // 4))).astype(np.int64)
    I, Q = oracle.qld(stack_from_series(x))
    R = oracle.amplitude(I, Q)[0, 0]
    expect = 2 * M * A * abs(math.sin(M * delta / 2) / (M * math.sin(delta / 2)))
    assert abs(R - expect) <= math.sqrt(2) * M + 1e-6
    assert 0.93 < expect / (2 * M * A) < 0.94


def test_on_bin_dft_equals_i_minus_iq_and_numpy_fft():
    rng = np.random.default_rng(5)
    f = rng.integers(0, 4096, size=(64, 3, 7)).astype(np.uint16)
    I, Q = oracle.qld(f)
    ref = np.fft.fft(f.astype(np.float64), axis=0)
    X = oracle.dft_bin(f, 16)
    assert np.abs(ref[16] - (I - 1j * Q)).max() < 1e-6
    assert np.abs(X - ref[16]).max() < 1e-6
    for k in (0, 1, 5, 31, 47, 63):
        assert np.abs(oracle.dft_bin(f, k) - ref[k]).max() < 1e-6


def test_dft_ragged_length_and_negative_bin():
    rng = np.random.default_rng(6)
    f = rng.integers(0, 256, size=(37, 2, 2)).astype(np.uint8)
    ref = np.fft.fft(f.astype(np.float64), axis=0)
    for k in (3, 9, -4):
        assert np.abs(oracle.dft_bin(f, k) - ref[k % 37]).max() < 1e-8


def test_linearity_and_cycle_permutation():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 1000, size=(32, 4, 4)).astype(np.uint16)
    y = rng.integers(0, 1000, size=(32, 4, 4)).astype(np.uint16)
    Ix, Qx = oracle.qld(x)
    Iy, Qy = oracle.qld(y)
    I, Q = oracle.qld((3 * x.astype(np.int64) + 2 * y).astype(np.uint16))
    assert (I == 3 * Ix + 2 * Iy).all() and (Q == 3 * Qx + 2 * Qy).all()
    perm = rng.permutation(8)
    xp = x.reshape(8, 4, 4, 4)[perm].reshape(32, 4, 4)
    Ip, Qp = oracle.qld(xp)
    assert (Ip == Ix).all() and (Qp == Qx).all()
    # Shuffling frames across phases does change the result (the test can fail).
    Is, Qs = oracle.qld(x[rng.permutation(32)])
    assert (Is != Ix).any() or (Qs != Qx).any()


def test_split_over_frames_and_phase_rotation():
    rng = np.random.default_rng(8)
    x = rng.integers(0, 65536, size=(23, 3, 5)).astype(np.uint16)
    I, Q = oracle.qld(x, phase0=2)
    I1, Q1 = oracle.qld(x[:10], phase0=2)
    I2, Q2 = oracle.qld(x[10:], phase0=12)
    assert (I1 + I2 == I).all() and (Q1 + Q2 == Q).all()
    # One step of phase0 rotates the quadratures: (I, Q) -> (-Q, I).
    Ir, Qr = oracle.qld(x, phase0=3)
    assert (Ir == -Q).all() and (Qr == I).all()


def test_overflow_edge_u16():
    # Largest window an int32 accumulator holds for 16-bit data: 32768 * 65535 < 2^31 <= 32769 * 65535.
    M = 32768
    series = np.tile(np.array([65535, 0, 0, 0], dtype=np.int64), M)
    I, Q = oracle.qld(stack_from_series(series))
    assert I[0, 0] == 65535 * M and I[0, 0] < 2 ** 31 and Q[0, 0] == 0


def test_brute_force_tiny_against_fft_definition():
    # 4 x 4 pixels: (I, Q) from the numpy FFT bin T/4 (a textbook routine).
    rng = np.random.default_rng(9)
    for T in (4, 8, 12, 64):
        f = rng.integers(0, 4096, size=(T, 4, 4)).astype(np.uint16)
        X = np.fft.fft(f.astype(np.float64), axis=0)[T // 4]
        I, Q = oracle.qld(f)
        assert (I == np.rint(X.real).astype(np.int64)).all()
        assert (Q == np.rint(-X.imag).astype(np.int64)).all()


def test_strided_views_match_contiguous():
    rng = np.random.default_rng(10)
    buf = rng.integers(0, 256, size=(12, 6, 20)).astype(np.uint8)
    view = buf[:, :, 3:14]
    I, Q = oracle.qld(view, 1)
    I2, Q2 = oracle.qld(np.ascontiguousarray(view), 1)
    assert (I == I2).all() and (Q == Q2).all()


def test_frame_stats():
    f = np.zeros((5, 3, 4), dtype=np.uint16)
    f[0] = 7
    f[1, 0, 0] = 4095
    f[2] = 4095
    f[3, 1, 2] = 65535
    s, n = oracle.frame_stats(f, 12)
    assert list(s) == [7 * 12, 4095, 4095 * 12, 65535, 0]
    assert list(n) == [0, 1, 12, 0, 0]
    s8, n8 = oracle.frame_stats(np.full((2, 2, 2), 255, np.uint8), 8)
    assert list(s8) == [1020, 1020] and list(n8) == [4, 4]


def test_amplitude_special_cases():
    I = np.array([7, -7, 0, 3, 3000, -2 ** 31 + 1, 2 ** 31 - 1, 0, 123456])
    Q = np.array([0, 0, 0, 4, 4000, 0, 2 ** 31 - 1, -9, 654321])
    R = oracle.amplitude(I, Q)
    assert list(R[:5]) == [7.0, 7.0, 0.0, 5.0, 5000.0]
    assert R[5] == 2 ** 31 - 1
    for i in range(len(I)):
        assert abs(R[i] - math.hypot(float(I[i]), float(Q[i]))) <= 1e-15 * R[i]


def test_window_brute_force():
    rng = np.random.default_rng(11)
    cycles = [rng.integers(0, 4096, size=(4, 3, 3)).astype(np.uint16) for _ in range(9)]
    out = list(oracle.window_series(cycles, 4, resets=[6]))
    for c, (I, Q, n) in enumerate(out):
        lo = 6 if c >= 6 else max(0, c - 3)
        ref = oracle.qld(np.concatenate(cycles[lo:c + 1]))
        assert n == c - lo + 1 and (I == ref[0]).all() and (Q == ref[1]).all()


def test_window_sinusoid_closed_form():
    # Inside any window of n cycles a pure sinusoid gives I = 2 n a, Q = 2 n b.
    a, b, c = 3, -4, 50
    cyc = np.array([c + a, c + b, c - a, c - b], dtype=np.uint16)[:, None, None]
    for I, Q, n in oracle.window_series([cyc] * 10, 6):
        assert I[0, 0] == 2 * n * a and Q[0, 0] == 2 * n * b


def test_frame_window_sinusoid_closed_form():
    # Every full period of a pure sinusoid adds (2a, 2b) whatever frame it
    # starts on, so a window of n frames (n a multiple of 4) gives I = 2 (n/4) a.
    a, b, c, M = 5, -3, 40, 3
    per = [c + a, c + b, c - a, c - b]
    frames = [np.full((2, 2), per[t % 4], dtype=np.uint16) for t in range(30)]
    for f, (I, Q, n) in enumerate(oracle.frame_window_series(frames, M)):
        assert n == min(f + 1, 4 * M)
        if n % 4 == 0:
            assert (I == 2 * (n // 4) * a).all() and (Q == 2 * (n // 4) * b).all(), f


def test_frame_window_impulse_enters_and_leaves():
    # One frame of value v at t0: it contributes v * (c, s)(phase of t0) while
    # inside the window of 4M frames, and nothing once it has left.
    M, t0, v, p0 = 2, 5, 7, 3
    frames = [np.zeros((1, 1), dtype=np.uint16) for _ in range(20)]
    frames[t0][0, 0] = v
    c, s = oracle.reference_tables()
    ph = (p0 + t0) % 4
    for f, (I, Q, n) in enumerate(oracle.frame_window_series(frames, M, phase0=p0)):
        inside = t0 <= f < t0 + 4 * M
        assert I[0, 0] == (v * c[ph] if inside else 0) and Q[0, 0] == (v * s[ph] if inside else 0), f


def test_frame_window_matches_cycle_window_and_reset():
    rng = np.random.default_rng(12)
    frames = [rng.integers(0, 4096, size=(3, 4)).astype(np.uint16) for _ in range(24)]
    cycles = [np.stack(frames[4 * k:4 * k + 4]) for k in range(6)]
    fw = list(oracle.frame_window_series(frames, 2))
    cw = list(oracle.window_series(cycles, 2))
    for k in range(6):                       # cycle-aligned frames: the same window
        assert (fw[4 * k + 3][0] == cw[k][0]).all() and (fw[4 * k + 3][1] == cw[k][1]).all()
    # A reset at frame r with phase p equals a fresh window started there.
    r, p = 9, 2
    with_reset = list(oracle.frame_window_series(frames, 2, resets={r: p}))
    fresh = list(oracle.frame_window_series(frames[r:], 2, phase0=p))
    for f in range(r, 24):
        assert (with_reset[f][0] == fresh[f - r][0]).all() and (with_reset[f][1] == fresh[f - r][1]).all()
        assert with_reset[f][2] == fresh[f - r][2]


def test_lockin_ratio_quarter_is_the_integer_lockin():
    # p/q = 1/4 with t0 = phase0 reduces to the four-sample QLD: X = I - iQ.
    rng = np.random.default_rng(21)
    st = rng.integers(0, 4096, size=(23, 3, 5)).astype(np.uint16)
    for p0 in range(4):
        I, Q = oracle.qld(st, p0)
        X = oracle.lockin_ratio(st, 1, 4, p0)
        assert np.allclose(X.real, I, atol=1e-9) and np.allclose(X.imag, -Q, atol=1e-9)
        X5 = oracle.lockin_ratio(st, 5, 4, p0)            # p is taken mod q
        assert np.allclose(X5, X, atol=1e-9)


def test_lockin_ratio_matches_fft_and_rejects_other_frequencies():
    rng = np.random.default_rng(22)
    T = 60
    st = rng.integers(0, 255, size=(T, 2, 3)).astype(np.uint8)
    F = np.fft.fft(st.astype(np.float64), axis=0)
    for k in (0, 1, 7, 15, 59):                           # q = T: the DFT bin k
        assert np.allclose(oracle.lockin_ratio(st, k, T), F[k], atol=1e-8)
    # A source at 3/20 of the sampling rate, seen at 7/20 over 60 frames (three
    # whole beat periods): nothing; at its own frequency: amplitude A T / 2.
    A, t = 50.0, np.arange(T)
    src = np.rint(100 + A * np.cos(2 * np.pi * 3 * t / 20)).astype(np.uint16)
    seq = stack_from_series(src)
    own = oracle.lockin_ratio(seq, 3, 20)[0, 0]
    other = oracle.lockin_ratio(seq, 7, 20)[0, 0]
    resid = src - (100 + A * np.cos(2 * np.pi * 3 * t / 20))  # rounding of the samples
    bound = np.abs(resid).sum()
    assert abs(abs(own) - A * T / 2) <= bound and abs(other) <= bound


def test_lockin_bank_is_the_full_fft_when_every_bin_is_asked():
    rng = np.random.default_rng(23)
    T = 24
    st = rng.integers(0, 4096, size=(T, 2, 3)).astype(np.uint16)
    X = oracle.lockin_bank(st, list(range(T)), T)
    assert np.allclose(X, np.fft.fft(st.astype(np.float64), axis=0), atol=1e-7)


def test_cnr_surround_matches_paper_example():
    g = read_kv("surround_fig_s.txt")
    src, surr = judges.square_masks((g["frame_h"], g["frame_w"]), 4, 4, g["source_side"])
    assert src.sum() == g["source_pixels"] and surr.sum() == g["surround_pixels"]
    assert surr.sum() == g["surround_squares"] * g["source_side"] ** 2
    assert not (src & surr).any()


def test_cnr_definition_values():
    img = np.zeros((14, 16))
    src, surr = judges.square_masks(img.shape, 4, 4, 4)
    img[surr] = np.tile([1.0, 3.0], 64)      # surround mean 2, RMS about the mean 1
    img[src] = 7.0
    assert abs(judges.cnr(img, src, surr) - 5.0) < 1e-12
    dsrc, dsur = judges.disk_masks((101, 101), 50, 50, 10)
    assert abs(dsur.sum() / dsrc.sum() - 8.0) < 0.2
    psrc, psur = judges.point_masks((20, 20), 10, 10)
    assert psrc.sum() == 9 and psur.sum() == 72


def test_nrmse():
    ref = np.array([3.0, 4.0])
    assert judges.nrmse(ref, ref) == 0.0
    assert abs(judges.nrmse(ref * 1.1, ref) - 0.1) < 1e-12
