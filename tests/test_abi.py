"""The C-ABI library: loads, exports every declared entry point, and rejects bad
arguments synchronously (no device is touched, so these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1511_03390_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qld.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+char\s*\*|qld_status|size_t|int32_t|int64_t)\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(q.lib, n), n
    assert sorted(q.EXPORTS) == names


def test_version_and_status_strings():
    assert "gfx950" in q.version()
    for st in range(13):
        assert q.lib.qld_status_str(st).startswith(b"QLD_")


def desc(H=4, W=4, rp=None, fs=None, dt=q.U16, bits=12):
    rp = W if rp is None else rp
    fs = H * rp if fs is None else fs
    return q.FrameDesc(H, W, rp, fs, dt, bits)


def acc(d, n=4, frames=1, I=1, Q=1):
    p = lambda v: ctypes.c_void_p(v) if v else None
    return q.lib.qld_accumulate(p(frames), ctypes.byref(d) if d is not None else None, n, 0, p(I), p(Q),
                                None, None, None)


def test_accumulate_argument_errors():
    assert q.lib.qld_accumulate(None, None, 4, 0, None, None, None, None, None) == q.E_INVAL
    assert acc(desc(dt=7)) == q.E_DTYPE
    assert acc(desc(dt=q.U8, bits=9)) == q.E_DTYPE
    assert acc(desc(bits=0)) == q.E_DTYPE
    assert acc(desc(rp=3)) == q.E_SHAPE
    assert acc(desc(fs=10)) == q.E_SHAPE
    assert acc(desc(H=-1)) == q.E_SHAPE
    assert acc(desc(), n=-1) == q.E_INVAL
    assert acc(desc(), frames=0) == q.E_INVAL
    assert acc(desc(), I=0) == q.E_INVAL
    # ceil(n/4) * (2^bits - 1) must stay below 2^31.
    assert acc(desc(bits=16), n=4 * 32769) == q.E_OVERFLOW
    assert acc(desc(bits=12), n=4 * 524417) == q.E_OVERFLOW
    assert b"overflow" in q.lib.qld_last_error()


def test_frame_stride_hint():
    # Sizes that are multiples of 64 KiB get a gap: 4 KiB from 2 MiB up
    # (1024 x 1024 and 2048 x 2048 uint16), 256 bytes below (1 MiB and less).
    assert q.frame_stride_hint(1024, 1024) == 1024 * 1024 + 2048
    assert q.frame_stride_hint(2048, 2048) == 2048 * 2048 + 2048
    assert q.frame_stride_hint(1024, 2048, dtype=q.U8) == 1024 * 2048 + 4096
    assert q.frame_stride_hint(256, 256) == 256 * 256 + 128
    assert q.frame_stride_hint(512, 512) == 512 * 512 + 128
    assert q.frame_stride_hint(1024, 1024, dtype=q.U8) == 1024 * 1024 + 256
    # Other sizes: rounded up to 256 bytes only.
    assert q.frame_stride_hint(2160, 2160) == 2160 * 2160          # 9 331 200 B, a multiple of 256
    assert q.frame_stride_hint(7, 13) == 128                        # 182 B -> 256 B
    assert q.frame_stride_hint(7, 13, row_pitch=16, dtype=q.U8) == 256
    assert q.frame_stride_hint(0, 5) == 0                           # empty frames need no stride
    for H, W, rp, dt in ((1024, 1024, 1024, q.U16), (480, 640, 704, q.U16), (33, 7, 7, q.U8)):
        fs = q.frame_stride_hint(H, W, row_pitch=rp, dtype=dt)
        eb = 2 if dt == q.U16 else 1
        assert fs >= H * rp and (fs * eb) % 256 == 0 and (fs * eb) % 65536 != 0
    assert q.frame_stride_hint(-1, 4) == 0
    assert q.frame_stride_hint(4, 4, row_pitch=3) == 0
    assert q.frame_stride_hint(4, 4, dtype=7) == 0


def test_read_probe_argument_errors():
    out = ctypes.c_void_p(1 << 20)
    assert q.lib.qld_read_probe(ctypes.c_void_p(1 << 20 | 8), 64, out, None) == q.E_ALIGN
    assert q.lib.qld_read_probe(ctypes.c_void_p(1 << 20), 65, out, None) == q.E_ALIGN
    assert q.lib.qld_read_probe(ctypes.c_void_p(1 << 20), -16, out, None) == q.E_ALIGN
    assert q.lib.qld_read_probe(ctypes.c_void_p(1 << 20), 64, None, None) == q.E_INVAL
    assert q.lib.qld_read_probe(None, 64, out, None) == q.E_INVAL


def test_empty_inputs_are_noops():
    assert acc(desc(), n=0, frames=0, I=0, Q=0) == q.OK
    assert acc(desc(H=0), frames=0, I=0, Q=0) == q.OK
    assert q.lib.qld_amplitude(None, None, 0, None, None) == q.OK
    assert q.lib.qld_amplitude(None, None, -1, None, None) == q.E_INVAL


def test_dft_and_window_argument_errors():
    d = desc()
    assert q.lib.dft_bin_baseline(ctypes.c_void_p(1), ctypes.byref(d), 0, 1, ctypes.c_void_p(1),
                                  ctypes.c_void_p(1), None) == q.E_SHAPE
    h = ctypes.c_void_p()
    assert q.lib.qld_window_create(ctypes.byref(d), 0, ctypes.byref(h)) == q.E_INVAL
    d16 = desc(bits=16)
    assert q.lib.qld_window_create(ctypes.byref(d16), 32769, ctypes.byref(h)) == q.E_OVERFLOW
    assert q.lib.qld_window_update(None, None, None, None, None, None, None) == q.E_INVAL
    assert q.lib.qld_window_bytes(ctypes.byref(d), 0) == 0
    # ring of int16 pairs (4 B/px/cycle) + I/Q (8 B/px); rows padded to 8 px.
    assert q.lib.qld_window_bytes(ctypes.byref(desc(H=3, W=5)), 10) == 10 * 3 * 8 * 4 + 3 * 8 * 8
    assert q.lib.qld_window_bytes(ctypes.byref(desc(H=3, W=8, bits=16)), 2) == 2 * 24 * 8 + 24 * 8


def test_server_argument_errors():
    assert q.lib.qld_server_create(1 << 20, 0, 0, ctypes.byref(ctypes.c_void_p())) == q.E_INVAL
    assert q.lib.qld_stream_submit(None, 1, None, 0, 0) == q.E_INVAL
    assert q.lib.qld_stream_poll(None, None, 0, None) == q.E_INVAL


def test_noalloc_scratch_limit_is_checked_before_any_launch():
    src = open(os.path.join(ROOT, "include", "qld.h")).read()
    m = re.search(r"#define QLD_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == q.NOALLOC_SCRATCH_BYTES
    # An unaligned 8-bit 1024 x 1024 x 257 stack with statistics needs
    # 4096 * 4 * 257 * 8 bytes of partials: more than the array holds, refused
    # synchronously (the pointers are never dereferenced).
    d = desc(H=1024, W=1024, dt=q.U8, bits=8)
    p = ctypes.c_void_p
    st = q.lib.qld_lockin_image_noalloc(p(1 << 20 | 1), ctypes.byref(d), 257, 0, p(1 << 21), p(1 << 22), None,
                                        p(1 << 23), p(1 << 24), None)
    assert st == q.E_NOMEM
    assert b"scratch" in q.lib.qld_last_error()
    assert q.lib.qld_lockin_image_noalloc(p(1 << 20), ctypes.byref(d), 0, 0, p(1 << 21), p(1 << 22), None,
                                          None, None, None) == q.E_SHAPE
