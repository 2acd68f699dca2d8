"""Training-data assignment (Sec. 3.2.2, Eqs. 3-5), plain FP64 NumPy: TEST
INFRASTRUCTURE ONLY.

  B1(pose, block j) = 1 when the SSIM loss between the render of every block and
                      the render without block j exceeds epsilon (Eq. 3);
  B2(pose, block j) = 1 when the pose's camera centre, normalised and contracted
                      (Eq. 2), lies in block j (Eq. 4);
  B = B1 or B2 (Eq. 5).

Readings (also listed in the design notes):
  * SSIM loss = 1 - SSIM, SSIM as defined by Wang et al. (2004) with the window
    of the 3DGS training code: an 11 x 11 Gaussian of standard deviation 1.5,
    normalised, applied per colour channel with zero padding outside the image;
    C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1); the image SSIM is the mean of
    the per-pixel map over pixels and channels;
  * Eq. 5's "+" on indicator values is a logical or.
"""
from __future__ import annotations

import math

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window():
    """Normalised 1-D Gaussian taps, offsets -5 .. 5."""
    r = WINDOW // 2
    w = np.array([math.exp(-(k * k) / (2.0 * SIGMA * SIGMA)) for k in range(-r, r + 1)])
    return w / w.sum()


def filter2d(img):
    """Zero-padded 'same' convolution of a 2-D image with the separable window."""
    w = gaussian_window()
    r = WINDOW // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    rows = np.zeros((H + 2 * r, W))
    for k in range(WINDOW):
        rows += w[k] * pad[:, k:k + W]
    out = np.zeros((H, W))
    for k in range(WINDOW):
        out += w[k] * rows[k:k + H, :]
    return out


def ssim_map(x, y):
    """Per-pixel SSIM of two single-channel images."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = filter2d(x), filter2d(y)
    sxx = filter2d(x * x) - mx * mx
    syy = filter2d(y * y) - my * my
    sxy = filter2d(x * y) - mx * my
    return ((2.0 * mx * my + C1) * (2.0 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(a, b):
    """Mean SSIM of two [3, H, W] images over pixels and channels."""
    return float(np.mean([ssim_map(a[c], b[c]).mean() for c in range(a.shape[0])]))


def assign(ssim_all_vs_without, cam_block, n_blocks, eps):
    """Eqs. 3-5.  ssim_all_vs_without [P, B]: SSIM between each pose's full render
    and its render without block j; cam_block [P]: block holding the contracted
    camera centre.  Returns (B1, B2, B) as bool [P, B]."""
    s = np.asarray(ssim_all_vs_without, np.float64)
    b1 = (1.0 - s) > eps
    b2 = np.zeros_like(b1)
    for p, j in enumerate(cam_block):
        b2[p, j] = True
    return b1, b2, b1 | b2
