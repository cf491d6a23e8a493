"""CPU oracle for quadrature lock-in discrimination (QLD) and its plain DFT baseline.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_1511_03390_amd`` and never imports it.

The arithmetic lives in ``qld_oracle.c`` and ``gen_oracle.c`` (plain C, built
with gcc -O2, no fast-math); this module loads them with ctypes and adds the
brute-force sliding window, which re-sums the stored history of frames at
every step.  ``oracle.learned`` holds the training-pair generator and the
denoiser (numpy, double precision).

Functions:
    qld(frames, phase0=0)            -> (I, Q) int64       (Methods, R(j,k))
    frame_stats(frames, bits)        -> (sum u64, sat u32)
    amplitude(I, Q)                  -> float64            (Methods, R(j,k))
    dft_bin(frames, k)               -> complex128         (Methods, Fourier map)
    window_series(cycles, M, resets) -> per-cycle (I, Q)   (Supplementary, sliding sequence)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "qld_oracle.c"), os.path.join(_HERE, "gen_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle's C sources into liboracle.so with gcc (always when force)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", *_SRCS, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_qld.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                   _i64p, _i64p, ctypes.c_int]
        lib.oracle_frame_stats.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                           _u64p, _u32p]
        lib.oracle_amplitude.argtypes = [_i64p, _i64p, ctypes.c_int64, _f64p]
        lib.oracle_amplitude.restype = None
        lib.oracle_dft_bin.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       _f64p, _f64p, ctypes.c_int]
        lib.oracle_lockin_ratio.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, _f64p, _f64p, ctypes.c_int]
        lib.oracle_reference_tables.argtypes = [_i64p, _i64p]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_philox4x32.argtypes = [u32p, u32p, ctypes.c_int, u32p]
        lib.oracle_philox4x32.restype = None
        lib.oracle_poisson_bounds.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_poisson_table.argtypes = [ctypes.c_double, u32p, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_poisson_invert.argtypes = [u32p, ctypes.c_int, ctypes.c_int32, ctypes.c_uint32]
        lib.oracle_poisson_invert.restype = ctypes.c_int32
        lib.oracle_gen_frames.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_gen_pixels.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def _frames_args(frames):
    """(pointer, elem, H, W, row_pitch, frame_stride, T) of a [T][H][W] numpy view."""
    a = np.asarray(frames)
    if a.ndim == 2:
        a = a[None]
    if a.dtype not in (np.uint8, np.uint16):
        raise TypeError("frames must be uint8 or uint16, got %s" % a.dtype)
    T, H, W = a.shape
    es = a.itemsize
    st = [s // es for s in a.strides]
    if a.strides[2] != es or any(s % es for s in a.strides):
        raise ValueError("innermost axis must be contiguous")
    if T == 0 or H == 0 or W == 0:
        ptr = 0
    else:
        ptr = a.__array_interface__["data"][0]
    return ptr, es, H, W, st[1], st[0], T, a


def threads() -> int:
    return int(os.environ.get("QLD_ORACLE_THREADS", "1"))


def reference_tables():
    c = (ctypes.c_int64 * 4)()
    s = (ctypes.c_int64 * 4)()
    if _load().oracle_reference_tables(c, s):
        raise RuntimeError("reference tables are not integers")
    return list(c), list(s)


def qld(frames, phase0: int = 0, n_threads: int | None = None):
    """Quadrature sums (I, Q) of every pixel, int64 [H][W]."""
    ptr, es, H, W, rp, fs, T, keep = _frames_args(frames)
    I = np.zeros((H, W), dtype=np.int64)
    Q = np.zeros((H, W), dtype=np.int64)
    if T and H and W:
        rc = _load().oracle_qld(ptr, es, H, W, rp, fs, T, int(phase0),
                                I.ctypes.data_as(_i64p), Q.ctypes.data_as(_i64p),
                                n_threads or threads())
        if rc:
            raise RuntimeError("oracle_qld failed (%d)" % rc)
    return I, Q


def frame_stats(frames, bits: int):
    """Per-frame (sum, count of samples equal to 2^bits - 1)."""
    ptr, es, H, W, rp, fs, T, keep = _frames_args(frames)
    s = np.zeros(T, dtype=np.uint64)
    n = np.zeros(T, dtype=np.uint32)
    if T and H and W:
        _load().oracle_frame_stats(ptr, es, H, W, rp, fs, T, int(bits),
                                   s.ctypes.data_as(_u64p), n.ctypes.data_as(_u32p))
    return s, n


def amplitude(I, Q):
    """(I^2 + Q^2)^(1/2) in double, from exact integer sums of squares."""
    I = np.ascontiguousarray(I, dtype=np.int64)
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    out = np.zeros(I.shape, dtype=np.float64)
    _load().oracle_amplitude(I.ctypes.data_as(_i64p), Q.ctypes.data_as(_i64p), I.size,
                             out.ctypes.data_as(_f64p))
    return out


def dft_bin(frames, k: int, n_threads: int | None = None):
    """X_k of every pixel's series (N = T), complex128 [H][W]."""
    ptr, es, H, W, rp, fs, T, keep = _frames_args(frames)
    re = np.zeros((H, W))
    im = np.zeros((H, W))
    if T and H and W:
        rc = _load().oracle_dft_bin(ptr, es, H, W, rp, fs, T, int(k),
                                    re.ctypes.data_as(_f64p), im.ctypes.data_as(_f64p),
                                    n_threads or threads())
        if rc:
            raise RuntimeError("oracle_dft_bin failed (%d)" % rc)
    return re + 1j * im


def lockin_ratio(frames, p: int, q: int, t0: int = 0, n_threads: int | None = None):
    """Lock-in of every pixel's series at frequency ratio p/q (time of frame 0:
    t0), complex128 [H][W]: X = I - iQ with the cos/sin reference tables."""
    ptr, es, H, W, rp, fs, T, keep = _frames_args(frames)
    re = np.zeros((H, W))
    im = np.zeros((H, W))
    if T and H and W:
        rc = _load().oracle_lockin_ratio(ptr, es, H, W, rp, fs, T, int(p), int(q), int(t0),
                                         re.ctypes.data_as(_f64p), im.ctypes.data_as(_f64p), n_threads or threads())
        if rc:
            raise RuntimeError("oracle_lockin_ratio failed (%d)" % rc)
    return re + 1j * im


def lockin_bank(frames, p_list, q: int, t0: int = 0):
    """Lock-ins at ratios p_f / q for every f (the bank is one lock-in per
    frequency), complex128 [F][H][W]."""
    return np.stack([lockin_ratio(frames, p, q, t0) for p in p_list], axis=0)


def frame_window_series(frames, M: int, phase0: int = 0, resets=None):
    """Per-frame sliding window (Supplementary, sliding sequence): after frame
    f the window holds frames max(r, f - 4M + 1) .. f, r the latest reset at or
    before f, and frame f has lock-in phase (p_r + f - r) mod 4 where p_r is
    the phase given at that reset (phase0 for r = 0).  (I, Q) by re-summing the
    stored frames with the lock-in definition; yields (I, Q, n_in_window).

    ``frames``: sequence of [H][W] arrays.  ``resets``: {frame index: phase of
    that frame}.
    """
    resets = dict(resets or {})
    history = []
    start, p_start = 0, int(phase0) % 4
    for f, fr in enumerate(frames):
        history.append(np.asarray(fr))
        if f in resets:
            start, p_start = f, int(resets[f]) % 4
        lo = max(start, f - 4 * M + 1)
        stack = np.stack(history[lo:f + 1], axis=0)
        I, Q = qld(stack, (p_start + lo - start) % 4)
        yield I, Q, f - lo + 1


def window_series(cycles, M: int, resets=()):
    """Sliding-window (I, Q) after every cycle, by re-summing the stored history.

    ``cycles``: sequence of [4][H][W] frame groups (phases 0..3).  After cycle
    c the window holds cycles max(r, c - M + 1) .. c, where r is the latest
    reset at or before c (a reset at cycle r discards everything before r).
    Yields (I, Q, n_in_window) per cycle.  No running sums are kept, so the
    result never depends on subtracting old cycles.
    """
    resets = sorted(set(int(r) for r in resets))
    history = []
    start = 0
    for c, cyc in enumerate(cycles):
        history.append(np.asarray(cyc))
        if c in resets:
            start = c
        lo = max(start, c - M + 1)
        stack = np.concatenate(history[lo:c + 1], axis=0)
        I, Q = qld(stack, 0)
        yield I, Q, c - lo + 1
