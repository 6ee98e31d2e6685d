"""Pins of the image-quality metrics used by the closed-form field studies."""

import numpy as np

from image_metrics import mse, psnr, ssim, to_8bit


def test_psnr_of_a_known_error():
    a = np.zeros((20, 20, 3), np.uint8)
    b = a.copy()
    b[::2] = 10                      # half the pixels off by 10: MSE = 50
    assert mse(a, b) == 50.0
    assert abs(psnr(a, b) - 10 * np.log10(255 ** 2 / 50.0)) < 1e-12
    assert psnr(a, a) == float("inf")


def test_ssim_identity_symmetry_and_constant_images():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 256, (40, 50, 3)).astype(np.uint8)
    noise = rng.integers(-30, 31, a.shape)
    b = np.clip(a.astype(int) + noise, 0, 255).astype(np.uint8)
    c = np.clip(a.astype(int) + 3 * noise, 0, 255).astype(np.uint8)
    assert abs(ssim(a, a) - 1.0) < 1e-12
    assert abs(ssim(a, b) - ssim(b, a)) < 1e-12
    assert 0.0 < ssim(a, c) < ssim(a, b) < 1.0
    # two constant images u, v: no variance, so SSIM = (2uv + C1) / (u^2 + v^2 + C1)
    u, v = 100.0, 140.0
    c1 = (0.01 * 255) ** 2
    A = np.full((30, 30, 3), u, np.uint8)
    B = np.full((30, 30, 3), v, np.uint8)
    assert abs(ssim(A, B) - (2 * u * v + c1) / (u * u + v * v + c1)) < 1e-9


def test_to_8bit_rounds_and_clips():
    x = np.array([[[0.0, 0.5, 1.2, 0.3], [1.0 / 255 * 0.49, 1.0 / 255 * 0.51, -0.1, 1.0]]])
    np.testing.assert_array_equal(to_8bit(x), [[[0, 128, 255], [0, 1, 0]]])
