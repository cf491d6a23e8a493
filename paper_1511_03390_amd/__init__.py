"""MI355X (gfx950) quadrature lock-in discrimination: Python binding of libqld.

Thin ctypes layer over the C ABI declared in ``include/qld.h``.  It only
marshals arguments (torch tensors -> device pointers, the current torch
stream -> hipStream_t); every step of the computation runs in the HIP
kernels of ``libqld.so``.  There is no fallback: if the library is missing
or fails to load, importing this package raises.

Build the library with ``python paper_1511_03390_amd/_build.py`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqld.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libqld.so is not built (%s); run python paper_1511_03390_amd/_build.py" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

# Status codes (qld_status).
OK, E_INVAL, E_DTYPE, E_SHAPE, E_ALIGN, E_OVERFLOW, E_NOMEM, E_BUDGET, E_AGAIN, E_STATE, E_GAP, E_DEVICE, E_IO = range(13)
U8, U16 = 1, 2
NOALLOC_SCRATCH_BYTES = 32 << 20      # QLD_NOALLOC_SCRATCH_BYTES
STREAM_PENDING, STREAM_ACTIVE, STREAM_CLOSED = 1, 2, 3
SERVER_KEEP_IQ = 1
MODE_PLAIN, MODE_LEARNED = 0, 1

# Every entry point the header declares (checked by the tests).
EXPORTS = (
    "qld_accumulate", "qld_lockin_image", "qld_lockin_image_noalloc", "qld_amplitude", "dft_bin_baseline", "dft_bin_baseline_f64", "qld_lockin_ratio", "qld_lockin_bank",
    "qld_window_bytes", "qld_window_create", "qld_window_update", "qld_window_reset",
    "qld_window_destroy", "qld_window_info", "qld_window_save", "qld_window_load",
    "qld_fwindow_bytes", "qld_fwindow_create", "qld_fwindow_update", "qld_fwindow_reset", "qld_fwindow_info",
    "qld_fwindow_destroy",
    "qld_server_create", "qld_server_stream_bytes", "qld_stream_open", "qld_stream_state",
    "qld_stream_set_denoiser", "qld_stream_submit", "qld_stream_submit_cycle", "qld_server_hold",
    "qld_server_set_max_inflight", "qld_stream_poll", "qld_stream_result_valid", "qld_stream_result_iq",
    "qld_server_drain", "qld_stream_close", "qld_server_destroy", "qld_server_stats",
    "qld_status_str", "qld_last_error", "qld_version", "qld_time_next_kernel", "qld_frame_stride_hint", "qld_read_probe",
    "qld_gen_pairs", "qld_denoise_prepare", "qld_denoise_target", "qld_clean_amplitude",
    "qld_judge_nrmse", "qld_judge_cnr", "qld_denoiser_param_count", "qld_denoiser_create",
    "qld_denoiser_info", "qld_denoiser_destroy", "qld_denoiser_set_params", "qld_denoiser_get_params", "qld_denoiser_get_grads",
    "qld_denoiser_tensor", "qld_denoiser_forward", "qld_denoiser_backward", "qld_denoiser_adam",
)


class QldError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.qld_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, _lib.qld_status_str(status).decode(), msg))


class FrameDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("row_pitch", ctypes.c_int64),
                ("frame_stride", ctypes.c_int64), ("dtype", ctypes.c_int), ("bits", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("stream_id", ctypes.c_int32), ("warm", ctypes.c_int32), ("cycle", ctypes.c_int64),
                ("t_arrival_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("amp", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("amp_plain", ctypes.c_void_p), ("gate", ctypes.c_float), ("learned", ctypes.c_int32),
                ("seq", ctypes.c_int64)]


_vp, _i32, _i64, _u64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
_dp = ctypes.POINTER(FrameDesc)


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("qld_accumulate", ctypes.c_int, _vp, _dp, _i32, _i32, _vp, _vp, _vp, _vp, _vp)
_sig("qld_lockin_image", ctypes.c_int, _vp, _dp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("qld_lockin_image_noalloc", ctypes.c_int, _vp, _dp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("qld_amplitude", ctypes.c_int, _vp, _vp, _i64, _vp, _vp)
_sig("dft_bin_baseline", ctypes.c_int, _vp, _dp, _i32, _i32, _vp, _vp, _vp)
_sig("dft_bin_baseline_f64", ctypes.c_int, _vp, _dp, _i32, _i32, _vp, _vp, _vp)
_sig("qld_window_bytes", _sz, _dp, _i32)
_sig("qld_window_create", ctypes.c_int, _dp, _i32, ctypes.POINTER(_vp))
_sig("qld_window_update", ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32), _vp)
_sig("qld_window_reset", ctypes.c_int, _vp)
_sig("qld_window_destroy", ctypes.c_int, _vp)
_sig("qld_window_info", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64))
_sig("qld_window_save", ctypes.c_int, _vp, ctypes.c_char_p)
_sig("qld_lockin_ratio", ctypes.c_int, _vp, _dp, _i32, _i32, _i32, _i32, _vp, _vp, _vp)
_sig("qld_lockin_bank", ctypes.c_int, _vp, _dp, _i32, _i32, ctypes.POINTER(_i32), _i32, _i32, _vp, _vp, _vp)
_sig("qld_fwindow_bytes", _sz, _dp, _i32)
_sig("qld_fwindow_create", ctypes.c_int, _dp, _i32, _i32, ctypes.POINTER(_vp))
_sig("qld_fwindow_update", ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32), _vp)
_sig("qld_fwindow_reset", ctypes.c_int, _vp, _i32)
_sig("qld_fwindow_info", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64))
_sig("qld_fwindow_destroy", ctypes.c_int, _vp)
_sig("qld_window_load", ctypes.c_int, _vp, ctypes.c_char_p)
_sig("qld_server_create", ctypes.c_int, _sz, _i32, _i32, ctypes.POINTER(_vp))
_sig("qld_server_stream_bytes", _sz, _vp, _dp, _i32, _i32, _i32)
_sig("qld_stream_set_denoiser", ctypes.c_int, _vp, _i32, _vp, ctypes.c_float)
_sig("qld_denoiser_info", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_sig("qld_stream_open", ctypes.c_int, _vp, _dp, _i32, _i32, _i32, ctypes.POINTER(_i32))
_sig("qld_stream_state", ctypes.c_int, _vp, _i32, ctypes.POINTER(_i32))
_sig("qld_stream_submit", ctypes.c_int, _vp, _i32, _vp, _i64, _u64)
_sig("qld_stream_submit_cycle", ctypes.c_int, _vp, _i32, _vp, _i64, _u64)
_sig("qld_server_hold", ctypes.c_int, _vp, _i32)
_sig("qld_server_set_max_inflight", ctypes.c_int, _vp, _i32)
_sig("qld_stream_result_valid", ctypes.c_int, _vp, ctypes.POINTER(Result), ctypes.POINTER(_i32))
_sig("qld_stream_poll", ctypes.c_int, _vp, ctypes.POINTER(Result), _i32, ctypes.POINTER(_i32))
_sig("qld_stream_result_iq", ctypes.c_int, _vp, ctypes.POINTER(Result), ctypes.POINTER(_vp),
     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp))
_sig("qld_server_drain", ctypes.c_int, _vp)
_sig("qld_stream_close", ctypes.c_int, _vp, _i32)
_sig("qld_server_destroy", ctypes.c_int, _vp)
_sig("qld_server_stats", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
     ctypes.POINTER(_i32), ctypes.POINTER(_sz))
_sig("qld_status_str", ctypes.c_char_p, ctypes.c_int)
_sig("qld_last_error", ctypes.c_char_p)
_sig("qld_version", ctypes.c_char_p)
_sig("qld_time_next_kernel", ctypes.c_int, _vp, _vp)
_sig("qld_frame_stride_hint", _i64, _i32, _i32, _i64, ctypes.c_int)
_sig("qld_read_probe", ctypes.c_int, _vp, _i64, _vp, _vp)
_fp = ctypes.POINTER(ctypes.c_float)
_sig("qld_gen_pairs", ctypes.c_int, _vp, _vp, _i32, _i32, _i32, _i32, _i32, ctypes.c_uint32, ctypes.c_uint64, _i32,
     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("qld_denoise_prepare", ctypes.c_int, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp)
_sig("qld_denoise_target", ctypes.c_int, _vp, _vp, _vp, _i32, _vp, _i32, _i32, _i32, _vp, _vp)
_sig("qld_clean_amplitude", ctypes.c_int, _vp, _vp, _i32, _i32, _i32, _vp, _vp)
_sig("qld_judge_nrmse", ctypes.c_int, _vp, _vp, _vp, _i32, _i64, _vp, _vp)
_sig("qld_judge_cnr", ctypes.c_int, _vp, _vp, _i32, _i64, _vp, _vp)
_sig("qld_denoiser_param_count", _i32)
_sig("qld_denoiser_create", ctypes.c_int, _i32, _i32, _i32, ctypes.POINTER(_vp))
_sig("qld_denoiser_destroy", ctypes.c_int, _vp)
_sig("qld_denoiser_set_params", ctypes.c_int, _vp, _fp, _i32)
_sig("qld_denoiser_get_params", ctypes.c_int, _vp, _fp, _i32)
_sig("qld_denoiser_get_grads", ctypes.c_int, _vp, _fp, _i32)
_sig("qld_denoiser_tensor", ctypes.c_int, _vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_i64))
_sig("qld_denoiser_forward", ctypes.c_int, _vp, _vp, _i32, _vp, _vp, _vp)
_sig("qld_denoiser_backward", ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_float, _i32, _vp, _vp)
_sig("qld_denoiser_adam", ctypes.c_int, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp)

lib = _lib


class KernelTimer:
    """HIP events (from the HIP runtime, on the launch stream) around the main
    kernel of the next qld_accumulate / dft_bin_baseline / qld_lockin_ratio /
    qld_lockin_bank / qld_denoiser_forward call of this thread."""

    _hip = None

    def __init__(self):
        if KernelTimer._hip is None:
            h = ctypes.CDLL("libamdhip64.so")
            h.hipEventCreate.argtypes = [ctypes.POINTER(_vp)]
            h.hipEventDestroy.argtypes = [_vp]
            h.hipEventSynchronize.argtypes = [_vp]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), _vp, _vp]
            KernelTimer._hip = h
        self.start, self.stop = _vp(), _vp()
        if self._hip.hipEventCreate(ctypes.byref(self.start)) or self._hip.hipEventCreate(ctypes.byref(self.stop)):
            raise RuntimeError("hipEventCreate failed")

    def arm(self):
        _check(_lib.qld_time_next_kernel(self.start, self.stop), "qld_time_next_kernel")

    def ms(self):
        if self._hip.hipEventSynchronize(self.stop):
            raise RuntimeError("hipEventSynchronize failed")
        out = ctypes.c_float()
        if self._hip.hipEventElapsedTime(ctypes.byref(out), self.start, self.stop):
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def __del__(self):
        try:
            self._hip.hipEventDestroy(self.start)
            self._hip.hipEventDestroy(self.stop)
        except Exception:
            pass


def _check(st, where, ok=(OK,)):
    if st not in ok:
        raise QldError(st, where)
    return st


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_DT = {torch.uint8: (U8, 8), torch.int16: (U16, 16), torch.uint16: (U16, 16)}


def frame_desc(frames: torch.Tensor, bits: int | None = None) -> FrameDesc:
    """Descriptor of a [T][H][W] (or [H][W]) frame tensor; innermost stride must be 1."""
    if frames.dtype not in _DT:
        raise TypeError("frames must be uint8, int16 or uint16 (16-bit samples), got %s" % frames.dtype)
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    if frames.dim() != 3:
        raise ValueError("frames must be [T][H][W]")
    T, H, W = frames.shape
    if W > 1 and frames.stride(2) != 1:
        raise ValueError("frames must be contiguous along W")
    dt, nbits = _DT[frames.dtype]
    rp = frames.stride(1) if H > 1 else W
    fs = frames.stride(0) if T > 1 else H * rp
    return FrameDesc(int(H), int(W), int(rp), int(fs), dt, int(bits or nbits))


def frame_stride_hint(H, W, row_pitch=None, dtype=U16):
    """Frame stride (elements) to allocate an [T][H][row_pitch] stack with (qld_frame_stride_hint)."""
    return int(_lib.qld_frame_stride_hint(int(H), int(W), int(W if row_pitch is None else row_pitch), int(dtype)))


def read_probe(buf, out=None, stream=None):
    """XOR of every 8-byte word of a device tensor's bytes (a plain streaming read; qld_read_probe)."""
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=buf.device)
    _check(_lib.qld_read_probe(_ptr(buf), int(buf.numel() * buf.element_size()), _ptr(out), _stream(stream)),
           "qld_read_probe")
    return out


def accumulate(frames, I, Q, phase0=0, bits=None, frame_sum=None, frame_sat=None, stream=None):
    """I += sum over cycles (S0 - S2), Q += sum (S1 - S3) of a [T][H][W] device stack."""
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.qld_accumulate(_ptr(frames), ctypes.byref(d), int(n), int(phase0), _ptr(I), _ptr(Q),
                               _ptr(frame_sum), _ptr(frame_sat), _stream(stream)), "qld_accumulate")


def lockin_image(frames, I, Q, amp=None, phase0=0, bits=None, frame_sum=None, frame_sat=None, stream=None):
    """One image of a [T][H][W] device stack in one pass: I, Q (and amp, the
    statistics) overwritten."""
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.qld_lockin_image(_ptr(frames), ctypes.byref(d), int(n), int(phase0), _ptr(I), _ptr(Q), _ptr(amp),
                                 _ptr(frame_sum), _ptr(frame_sat), _stream(stream)), "qld_lockin_image")


def lockin_image_noalloc(frames, I, Q, amp=None, phase0=0, bits=None, frame_sum=None, frame_sat=None,
                         stream=None):
    """lockin_image through the entry point that allocates no device memory
    (its scratch is the library's fixed per-device array)."""
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.qld_lockin_image_noalloc(_ptr(frames), ctypes.byref(d), int(n), int(phase0), _ptr(I), _ptr(Q),
                                         _ptr(amp), _ptr(frame_sum), _ptr(frame_sat), _stream(stream)),
           "qld_lockin_image_noalloc")


def amplitude(I, Q, amp, stream=None):
    _check(_lib.qld_amplitude(_ptr(I), _ptr(Q), int(I.numel()), _ptr(amp), _stream(stream)), "qld_amplitude")


def lockin_ratio(frames, p, q, re, im, t0=0, bits=None, stream=None):
    """Lock-in at frequency ratio p/q (frames [T][H][W]); re/im float [H][W]; X = I - iQ."""
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.qld_lockin_ratio(_ptr(frames), ctypes.byref(d), int(n), int(p), int(q), int(t0), _ptr(re), _ptr(im),
                                 _stream(stream)), "qld_lockin_ratio")


def lockin_bank(frames, p_list, q, re=None, im=None, t0=0, bits=None, stream=None):
    """Bank of lock-ins at ratios p_f/q (frames [T][H][W]); returns re, im float [F][H][W]."""
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    F = len(p_list)
    if re is None:
        re = torch.empty((F, d.H, d.W), dtype=torch.float32, device=frames.device)
        im = torch.empty_like(re)
    arr = (_i32 * max(F, 1))(*[int(v) for v in p_list])
    _check(_lib.qld_lockin_bank(_ptr(frames), ctypes.byref(d), int(n), int(F), arr, int(q), int(t0), _ptr(re),
                                _ptr(im), _stream(stream)), "qld_lockin_bank")
    return re, im


def dft_bin_baseline(frames, k, re, im, bits=None, stream=None):
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.dft_bin_baseline(_ptr(frames), ctypes.byref(d), int(n), int(k), _ptr(re), _ptr(im),
                                 _stream(stream)), "dft_bin_baseline")


def dft_bin_baseline_f64(frames, k, re, im, bits=None, stream=None):
    """The single-bin DFT in double precision; re, im float64 [H][W]."""
    if re.dtype != torch.float64 or im.dtype != torch.float64:
        raise TypeError("re and im must be float64")
    d = frame_desc(frames, bits)
    n = frames.shape[0] if frames.dim() == 3 else 1
    _check(_lib.dft_bin_baseline_f64(_ptr(frames), ctypes.byref(d), int(n), int(k), _ptr(re), _ptr(im),
                                     _stream(stream)), "dft_bin_baseline_f64")


def lockin(frames, phase0=0, bits=None, stats=False, stream=None):
    """Convenience: fresh I, Q, amplitude (and per-frame stats) of a device stack (qld_lockin_image)."""
    T, H, W = frames.shape
    dev = frames.device
    I = torch.empty((H, W), dtype=torch.int32, device=dev)
    Q = torch.empty((H, W), dtype=torch.int32, device=dev)
    fsum = torch.empty(T, dtype=torch.int64, device=dev) if stats else None
    fsat = torch.empty(T, dtype=torch.int32, device=dev) if stats else None
    amp = torch.empty((H, W), dtype=torch.float32, device=dev)
    lockin_image(frames, I, Q, amp, phase0, bits, fsum, fsat, stream)
    return (I, Q, amp, fsum, fsat) if stats else (I, Q, amp)


class Window:
    """Sliding window of M cycles over frames of a fixed shape (device state)."""

    def __init__(self, H, W, M, dtype=torch.int16, bits=None):
        dt, nbits = _DT[dtype]
        self.desc = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        self.M = M
        self.H, self.W = H, W
        h = _vp()
        _check(_lib.qld_window_create(ctypes.byref(self.desc), int(M), ctypes.byref(h)), "qld_window_create")
        self._h = h

    @staticmethod
    def bytes(H, W, M, dtype=torch.int16, bits=None):
        dt, nbits = _DT[dtype]
        d = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        return int(_lib.qld_window_bytes(ctypes.byref(d), int(M)))

    def update(self, cycle_frames, I_out=None, Q_out=None, amp_out=None, stream=None):
        """Feed one cycle ([4][H][W] device tensor); returns warm (1 once M cycles are in)."""
        d = frame_desc(cycle_frames, self.desc.bits)
        if (d.H, d.W) != (self.H, self.W) or cycle_frames.shape[0] != 4:
            raise ValueError("cycle must be [4][%d][%d]" % (self.H, self.W))
        self.desc.row_pitch, self.desc.frame_stride = d.row_pitch, d.frame_stride
        warm = _i32()
        _check(_lib.qld_window_update(self._h, _ptr(cycle_frames), _ptr(I_out), _ptr(Q_out), _ptr(amp_out),
                                      ctypes.byref(warm), _stream(stream)), "qld_window_update")
        return warm.value

    def reset(self):
        _check(_lib.qld_window_reset(self._h), "qld_window_reset")

    def info(self):
        n, c = _i32(), _i64()
        _check(_lib.qld_window_info(self._h, ctypes.byref(n), ctypes.byref(c)), "qld_window_info")
        return n.value, c.value

    def save(self, path):
        _check(_lib.qld_window_save(self._h, str(path).encode()), "qld_window_save")

    def load(self, path):
        _check(_lib.qld_window_load(self._h, str(path).encode()), "qld_window_load")

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.qld_window_destroy(self._h), "qld_window_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameWindow:
    """Per-frame sliding window of the last 4 M frames (an image for every frame)."""

    def __init__(self, H, W, M, phase0=0, dtype=torch.int16, bits=None):
        dt, nbits = _DT[dtype]
        self.desc = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        self.H, self.W, self.M = H, W, M
        h = _vp()
        _check(_lib.qld_fwindow_create(ctypes.byref(self.desc), int(M), int(phase0), ctypes.byref(h)),
               "qld_fwindow_create")
        self._h = h

    @staticmethod
    def bytes(H, W, M, dtype=torch.int16, bits=None):
        dt, nbits = _DT[dtype]
        d = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        return int(_lib.qld_fwindow_bytes(ctypes.byref(d), int(M)))

    def update(self, frame, I_out=None, Q_out=None, amp_out=None, stream=None):
        """Feed one frame ([H][W] device tensor with contiguous rows); returns warm."""
        if tuple(frame.shape) != (self.H, self.W) or (self.H > 1 and frame.stride(0) != self.W) or \
                (self.W > 1 and frame.stride(1) != 1):
            raise ValueError("frame must be a contiguous [%d][%d] tensor" % (self.H, self.W))
        warm = _i32()
        _check(_lib.qld_fwindow_update(self._h, _ptr(frame), _ptr(I_out), _ptr(Q_out), _ptr(amp_out),
                                       ctypes.byref(warm), _stream(stream)), "qld_fwindow_update")
        return warm.value

    def reset(self, phase0=0):
        _check(_lib.qld_fwindow_reset(self._h, int(phase0)), "qld_fwindow_reset")

    def info(self):
        n, c = _i32(), _i64()
        _check(_lib.qld_fwindow_info(self._h, ctypes.byref(n), ctypes.byref(c)), "qld_fwindow_info")
        return n.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.qld_fwindow_destroy(self._h), "qld_fwindow_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server for many camera streams (see qld_server_* in qld.h)."""

    def __init__(self, hbm_budget_bytes, out_slots=8, keep_iq=False):
        h = _vp()
        _check(_lib.qld_server_create(int(hbm_budget_bytes), int(out_slots), SERVER_KEEP_IQ if keep_iq else 0,
                                      ctypes.byref(h)), "qld_server_create")
        self._h = h
        self.shapes = {}

    def stream_bytes(self, H, W, M, M_short=0, dtype=torch.int16, bits=None, mode=MODE_PLAIN):
        dt, nbits = _DT[dtype]
        d = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        return int(_lib.qld_server_stream_bytes(self._h, ctypes.byref(d), int(M), int(M_short), int(mode)))

    def open(self, H, W, M, M_short=0, dtype=torch.int16, bits=None, mode=MODE_PLAIN):
        """Returns (stream_id, admitted_now)."""
        dt, nbits = _DT[dtype]
        d = FrameDesc(int(H), int(W), int(W), int(H) * int(W), dt, int(bits or nbits))
        sid = _i32()
        st = _check(_lib.qld_stream_open(self._h, ctypes.byref(d), int(M), int(M_short), int(mode),
                                         ctypes.byref(sid)), "qld_stream_open", ok=(OK, E_AGAIN))
        self.shapes[sid.value] = (H, W)
        return sid.value, st == OK

    def set_denoiser(self, sid, denoiser, gate_threshold=0.05):
        """Attach a Denoiser (same H x W as the stream) to a LEARNED stream."""
        _check(_lib.qld_stream_set_denoiser(self._h, int(sid), denoiser._h, float(gate_threshold)),
               "qld_stream_set_denoiser")

    def state(self, sid):
        s = _i32()
        _check(_lib.qld_stream_state(self._h, int(sid), ctypes.byref(s)), "qld_stream_state")
        return s.value

    def submit(self, sid, frame, index, t_arrival_ns):
        """frame: host numpy array [H][W] (uint8 / uint16), C-contiguous.  Returns the status."""
        if not frame.flags["C_CONTIGUOUS"]:
            raise ValueError("frame must be C-contiguous")
        return _check(_lib.qld_stream_submit(self._h, int(sid), ctypes.c_void_p(frame.ctypes.data), int(index),
                                             int(t_arrival_ns)), "qld_stream_submit", ok=(OK, E_GAP, E_AGAIN))

    def submit_cycle(self, sid, frames, first_index, t_arrival_ns):
        """frames: host numpy array [4][H][W] (uint8 / uint16), C-contiguous, the
        frames first_index .. first_index + 3 (first_index a multiple of 4)."""
        if not frames.flags["C_CONTIGUOUS"]:
            raise ValueError("frames must be C-contiguous")
        return _check(_lib.qld_stream_submit_cycle(self._h, int(sid), ctypes.c_void_p(frames.ctypes.data),
                                                   int(first_index), int(t_arrival_ns)),
                      "qld_stream_submit_cycle", ok=(OK, E_GAP, E_AGAIN))

    def hold(self, on=True):
        _check(_lib.qld_server_hold(self._h, 1 if on else 0), "qld_server_hold")

    def set_max_inflight(self, n):
        _check(_lib.qld_server_set_max_inflight(self._h, int(n)), "qld_server_set_max_inflight")

    def result_valid(self, res):
        v = _i32()
        _check(_lib.qld_stream_result_valid(self._h, ctypes.byref(res), ctypes.byref(v)), "qld_stream_result_valid")
        return bool(v.value)

    def poll(self, max_results=256):
        buf = (Result * max_results)()
        n = _i32()
        _check(_lib.qld_stream_poll(self._h, buf, int(max_results), ctypes.byref(n)), "qld_stream_poll")
        return [buf[i] for i in range(n.value)]

    def result_iq(self, res):
        ptrs = [_vp() for _ in range(4)]
        _check(_lib.qld_stream_result_iq(self._h, ctypes.byref(res), *[ctypes.byref(p) for p in ptrs]),
               "qld_stream_result_iq")
        return [p.value for p in ptrs]

    def drain(self):
        _check(_lib.qld_server_drain(self._h), "qld_server_drain")

    def close_stream(self, sid):
        _check(_lib.qld_stream_close(self._h, int(sid)), "qld_stream_close")

    def stats(self):
        b, c, m, u = _i64(), _i64(), _i32(), _sz()
        _check(_lib.qld_server_stats(self._h, ctypes.byref(b), ctypes.byref(c), ctypes.byref(m), ctypes.byref(u)),
               "qld_server_stats")
        return dict(batches=b.value, cycles=c.value, max_streams_in_batch=m.value, bytes_in_use=u.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.qld_server_destroy(self._h), "qld_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(int(s) for s in shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2, "strides": None}


def device_view(ptr, shape, dtype, device=None):
    """Wrap a device pointer owned by libqld as a torch tensor (no copy, no ownership)."""
    typestr = {torch.float32: "<f4", torch.int32: "<i4"}[dtype]
    dev = device or torch.device("cuda", torch.cuda.current_device())
    return torch.as_tensor(_DeviceArray(ptr, shape, typestr), device=dev)


# ---------------------------------------------------------------------------
# Learned short-window path
# ---------------------------------------------------------------------------

def _host_f64(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, ctypes.c_void_p(a.ctypes.data)


def gen_pairs(mask, rates, M_short, M_long, tile0, seed, bits=12, stream=None):
    """Training pairs of n tiles: mask device uint8 [n][H][W], rates host [n][2][4].
    Returns device tensors (I_S, Q_S, I_L, Q_L, sum_S, sum_L, psum_S, psum_L):
    the per-pixel sample sums psum_* hold uint32 values in int32 tensors."""
    n, H, W = mask.shape
    dev = mask.device
    outs = [torch.empty((n, H, W), dtype=torch.int32, device=dev) for _ in range(4)]
    sums = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(2)]
    psums = [torch.empty((n, H, W), dtype=torch.int32, device=dev) for _ in range(2)]
    keep, rp = _host_f64(rates)
    _check(_lib.qld_gen_pairs(_ptr(mask), rp, int(n), int(H), int(W), int(M_short), int(M_long), int(tile0),
                              int(seed), int(bits), *[_ptr(o) for o in outs], _ptr(sums[0]), _ptr(sums[1]),
                              _ptr(psums[0]), _ptr(psums[1]), _stream(stream)), "qld_gen_pairs")
    return (*outs, *sums, *psums)


def denoise_prepare(I_S, Q_S, psum_S, sum_S, M_S, stream=None):
    B, H, W = I_S.shape
    x = torch.empty((B, H, W, 2), dtype=torch.float32, device=I_S.device)
    scale = torch.empty(B, dtype=torch.float32, device=I_S.device)
    _check(_lib.qld_denoise_prepare(_ptr(I_S), _ptr(Q_S), _ptr(psum_S), _ptr(sum_S), int(M_S), int(B), int(H), int(W),
                                    _ptr(x), _ptr(scale), _stream(stream)), "qld_denoise_prepare")
    return x, scale


def denoise_target(I_L, Q_L, psum_L, M_L, scale, stream=None):
    B, H, W = I_L.shape
    t = torch.empty((B, H, W), dtype=torch.float32, device=I_L.device)
    _check(_lib.qld_denoise_target(_ptr(I_L), _ptr(Q_L), _ptr(psum_L), int(M_L), _ptr(scale), int(B), int(H), int(W),
                                   _ptr(t), _stream(stream)), "qld_denoise_target")
    return t


def clean_amplitude(mask, rates, stream=None):
    B, H, W = mask.shape
    a = torch.empty((B, H, W), dtype=torch.float32, device=mask.device)
    keep, rp = _host_f64(rates)
    _check(_lib.qld_clean_amplitude(_ptr(mask), rp, int(B), int(H), int(W), _ptr(a), _stream(stream)),
           "qld_clean_amplitude")
    return a


def judge_nrmse(x, ref, scale=None, stream=None):
    B = x.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=x.device)
    _check(_lib.qld_judge_nrmse(_ptr(x), _ptr(scale), _ptr(ref), int(B), int(x[0].numel()), _ptr(out),
                                _stream(stream)), "qld_judge_nrmse")
    return out


def judge_cnr(img, labels, stream=None):
    B = img.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=img.device)
    _check(_lib.qld_judge_cnr(_ptr(img), _ptr(labels), int(B), int(img[0].numel()), _ptr(out), _stream(stream)),
           "qld_judge_cnr")
    return out


TENSORS = {"x0": 0, "a1": 1, "a2": 2, "a3": 3, "y": 4, "dz3": 5, "dz2": 6, "pool": 7, "gate": 8, "loss": 9, "dz1": 10}


class Denoiser:
    """The learned short-window denoiser (device weights, Adam state, activations)."""

    def __init__(self, H, W, max_batch):
        h = _vp()
        _check(_lib.qld_denoiser_create(int(H), int(W), int(max_batch), ctypes.byref(h)), "qld_denoiser_create")
        self._h, self.H, self.W, self.max_batch = h, H, W, max_batch
        self.n_params = int(_lib.qld_denoiser_param_count())

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params
        _check(_lib.qld_denoiser_set_params(self._h, a.ctypes.data_as(_fp), int(a.size)), "qld_denoiser_set_params")

    def get_params(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.qld_denoiser_get_params(self._h, a.ctypes.data_as(_fp), int(a.size)), "qld_denoiser_get_params")
        return a

    def get_grads(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.qld_denoiser_get_grads(self._h, a.ctypes.data_as(_fp), int(a.size)), "qld_denoiser_get_grads")
        return a

    def tensor(self, name):
        p, n = _vp(), _i64()
        _check(_lib.qld_denoiser_tensor(self._h, TENSORS[name], ctypes.byref(p), ctypes.byref(n)), "qld_denoiser_tensor")
        return p.value, n.value

    def forward(self, x, y=None, gate=None, stream=None):
        _check(_lib.qld_denoiser_forward(self._h, _ptr(x), int(x.shape[0]), _ptr(y), _ptr(gate), _stream(stream)),
               "qld_denoiser_forward")

    def backward(self, t, e_a=None, e_b=None, gate_weight=1.0, loss=None, stream=None):
        _check(_lib.qld_denoiser_backward(self._h, _ptr(t), _ptr(e_a), _ptr(e_b), float(gate_weight),
                                          int(t.shape[0]), _ptr(loss), _stream(stream)), "qld_denoiser_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.qld_denoiser_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
               "qld_denoiser_adam")

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.qld_denoiser_destroy(self._h), "qld_denoiser_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bf16_view(ptr, count, device=None):
    """float32 copy of a libqld bfloat16 device buffer (bits widened by 16)."""
    raw = device_view(ptr, ((count + 1) // 2,), torch.int32, device)
    lo = raw & 0xFFFF
    hi = (raw >> 16) & 0xFFFF
    words = torch.stack([lo, hi], dim=-1).reshape(-1)[:count]
    return (words << 16).view(torch.float32)


def version():
    return _lib.qld_version().decode()
