"""Helpers for the GPU tests: device upload of numpy stacks and ulp distance."""
import sys

import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(a):
    """numpy uint8/uint16 array (any strides along the outer axes) -> cuda tensor with the same bits."""
    a = np.asarray(a)
    if a.dtype == np.uint16:
        t = torch.from_numpy(np.ascontiguousarray(a).view(np.int16))
    elif a.dtype == np.uint8:
        t = torch.from_numpy(np.ascontiguousarray(a))
    else:
        raise TypeError(a.dtype)
    return t.cuda()


def to_host_u16(t):
    a = t.cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a


def ulp32(x):
    """Spacing of float32 at |x| (x in float64)."""
    x = np.abs(np.asarray(x, dtype=np.float64)).astype(np.float32)
    return np.spacing(x).astype(np.float64)


def amp_ulps(amp32, amp64):
    amp32 = np.asarray(amp32, dtype=np.float64)
    u = ulp32(amp64)
    u = np.where(u == 0, np.spacing(np.float32(0)), u)
    return np.abs(amp32 - amp64) / u


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
