"""Image-quality metrics of the closed-form field studies, on 8-bit RGB
images as the paper reports them (PSNR = 10 log10(255^2 / MSE)).

SSIM follows Wang, Bovik, Sheikh and Simoncelli (2004): an 11-tap Gaussian
window of standard deviation 1.5, K1 = 0.01, K2 = 0.03, L = 255, computed
per channel over the window positions that lie inside the image and
averaged."""

from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter


def to_8bit(rgba: np.ndarray) -> np.ndarray:
    """Premultiplied RGBA in [0,1] over a black background -> uint8 RGB."""
    rgb = np.clip(np.asarray(rgba, dtype=np.float64)[..., :3], 0.0, 1.0)
    return np.rint(rgb * 255.0).astype(np.uint8)


def mse(a: np.ndarray, b: np.ndarray) -> float:
    d = a.astype(np.float64) - b.astype(np.float64)
    return float((d * d).mean())


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    m = mse(a, b)
    return float("inf") if m == 0.0 else 10.0 * np.log10(255.0 ** 2 / m)


def ssim(a: np.ndarray, b: np.ndarray) -> float:
    a = a.astype(np.float64)
    b = b.astype(np.float64)
    c1, c2 = (0.01 * 255.0) ** 2, (0.03 * 255.0) ** 2
    r = 5                                   # 11-tap window: truncate at 5 / 1.5 sigma
    vals = []
    for ch in range(a.shape[-1]):
        x, y = a[..., ch], b[..., ch]
        filt = lambda t: gaussian_filter(t, 1.5, truncate=r / 1.5, mode="constant")
        mx, my = filt(x), filt(y)
        sxx = filt(x * x) - mx * mx
        syy = filt(y * y) - my * my
        sxy = filt(x * y) - mx * my
        s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        vals.append(s[r:-r, r:-r].mean())
    return float(np.mean(vals))
