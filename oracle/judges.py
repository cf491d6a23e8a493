"""Image-quality judges: contrast-to-noise ratio and normalized RMS error.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Double precision.

CNR follows the paper's Eq. CNR (Methods, "Estimation of contrast-to-noise
ratio"): the source mean minus the surround mean, divided by the RMS of the
surround about the surround mean.  For an m x m source the surround is the
m-pixel-wide square ring around it, 8 m^2 pixels (figure of a 14 x 16 frame
with a 4 x 4 source and a surround of eight 4 x 4 squares).  The paper defines
only square sources; the other shapes below keep the same 8x area ratio.
"""
from __future__ import annotations

import numpy as np


def square_masks(shape, y0, x0, h, w=None):
    """Source (h x w at y0, x0) and its ring: the (3h x 3w) box minus the source,
    clipped to the frame."""
    w = h if w is None else w
    H, W = shape
    src = np.zeros(shape, dtype=bool)
    src[y0:y0 + h, x0:x0 + w] = True
    box = np.zeros(shape, dtype=bool)
    box[max(0, y0 - h):min(H, y0 + 2 * h), max(0, x0 - w):min(W, x0 + 2 * w)] = True
    return src, box & ~src


def disk_masks(shape, cy, cx, r):
    """Disk of radius r and the annulus r < d <= 3r (area 8 pi r^2)."""
    yy, xx = np.mgrid[0:shape[0], 0:shape[1]]
    d2 = (yy - cy) ** 2 + (xx - cx) ** 2
    src = d2 <= r * r
    return src, (d2 <= 9 * r * r) & ~src


def point_masks(shape, cy, cx):
    """Point source: the 3 x 3 block around (cy, cx) and its 3-px-wide ring (72 px)."""
    return square_masks(shape, cy - 1, cx - 1, 3, 3)


def cnr(image, src, surr):
    img = np.asarray(image, dtype=np.float64)
    s = img[src]
    r = img[surr]
    mr = r.mean()
    return float((s.mean() - mr) / np.sqrt(np.mean((r - mr) ** 2)))


def nrmse(x, ref):
    """RMS(x - ref) / RMS(ref)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.mean((x - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
