"""Pins of the data-assignment oracle (Sec. 3.2.2, Eqs. 3-5): SSIM against an
independent filter implementation and closed forms, assignment rules (no GPU)."""
import numpy as np
import scipy.ndimage

from oracle import assign as oas
from oracle import partition as opart


def test_window_is_normalised_symmetric_gaussian():
    w = oas.gaussian_window()
    assert w.shape == (11,) and abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w, w[::-1], rtol=0, atol=0)
    assert abs(w[6] / w[5] - np.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-15


def test_filter_matches_scipy_gaussian_filter_with_zero_padding():
    rng = np.random.default_rng(0)
    img = rng.random((37, 53))
    # scipy: same normalised taps (radius = int(truncate * sigma + 0.5) = 5), constant-0 boundary
    ref = scipy.ndimage.gaussian_filter(img, sigma=1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
    np.testing.assert_allclose(oas.filter2d(img), ref, rtol=0, atol=1e-14)


def test_ssim_identity_symmetry_and_range():
    rng = np.random.default_rng(1)
    a = rng.random((3, 24, 31))
    b = np.clip(a + rng.normal(0, 0.1, a.shape), 0, 1)
    assert abs(oas.ssim(a, a) - 1.0) < 1e-12
    assert abs(oas.ssim(a, b) - oas.ssim(b, a)) < 1e-12
    assert -1.0 <= oas.ssim(a, b) < 1.0


def test_ssim_of_constant_images_interior_closed_form():
    # away from the zero-padded border the window sees constants c1, c2:
    # sigma terms vanish, SSIM = (2 c1 c2 + C1) / (c1^2 + c2^2 + C1)
    H, W = 40, 40
    c1, c2 = 0.7, 0.4
    m = oas.ssim_map(np.full((H, W), c1), np.full((H, W), c2))
    want = (2 * c1 * c2 + oas.C1) / (c1 * c1 + c2 * c2 + oas.C1)
    np.testing.assert_allclose(m[5:-5, 5:-5], want, rtol=1e-12)


def test_ssim_structure_term_for_an_affine_copy():
    # y = a x + b on a pattern: inside, sigma_xy = a sigma_x^2, sigma_y^2 = a^2 sigma_x^2 (exactly, per window)
    rng = np.random.default_rng(2)
    x = rng.random((30, 30))
    y = 0.5 * x + 0.2
    m = oas.ssim_map(x, y)
    mx = oas.filter2d(x)
    sxx = oas.filter2d(x * x) - mx * mx
    my = 0.5 * mx + 0.2 * oas.filter2d(np.ones_like(x))
    syy = 0.25 * sxx
    sxy = 0.5 * sxx
    want = ((2 * mx * my + oas.C1) * (2 * sxy + oas.C2)) / ((mx * mx + my * my + oas.C1) * (sxx + syy + oas.C2))
    np.testing.assert_allclose(m[5:-5, 5:-5], want[5:-5, 5:-5], rtol=1e-9)


def test_assignment_rules():
    s = np.array([[1.0, 0.96, 0.90], [0.999, 0.5, 1.0]])
    b1, b2, b = oas.assign(s, cam_block=[2, 0], n_blocks=3, eps=0.05)
    np.testing.assert_array_equal(b1, [[False, False, True], [False, True, False]])
    np.testing.assert_array_equal(b2, [[False, False, True], [True, False, False]])
    np.testing.assert_array_equal(b, [[False, False, True], [True, True, False]])


def test_camera_block_by_contraction():
    # a camera centre far outside the foreground box lands in an outer block
    means = np.array([[-100.0, 100.0], [-100.0, 100.0], [0.0, 40.0]])
    p_min, p_max = opart.foreground_box(means, (-100.0, -100.0), (100.0, 100.0))
    far = np.array([[5000.0], [0.0], [60.0]])
    assert opart.block_ids(far, p_min, p_max, 6, 6)[0] % 6 == 5
    centre = np.array([[1.0], [1.0], [20.0]])
    assert opart.block_ids(centre, p_min, p_max, 6, 6)[0] in (2 * 6 + 3, 3 * 6 + 3)


# ---------------------------------------------------------------------------
# SSIM against closed forms with the constants written out (C1 = 0.01^2 =
# 0.0001, C2 = 0.03^2 = 0.0009) and window moments from SciPy's filter, so the
# oracle's own constants and formula are not reused
# ---------------------------------------------------------------------------
def _scipy_moments(x):
    f = lambda a: scipy.ndimage.gaussian_filter(a, sigma=1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
    mu = f(x)
    return mu, f(x * x) - mu * mu


def test_ssim_constant_images_literal_constants():
    H, W = 40, 40
    for c1, c2 in ((0.7, 0.4), (0.05, 0.0), (0.3, 0.3)):
        m = oas.ssim_map(np.full((H, W), c1), np.full((H, W), c2))
        want = (2 * c1 * c2 + 0.0001) / (c1 * c1 + c2 * c2 + 0.0001)
        np.testing.assert_allclose(m[5:-5, 5:-5], want, rtol=1e-12)


def test_ssim_affine_copy_closed_form_literal_constants():
    # y = a x + b: sigma_xy = a sigma^2, sigma_y^2 = a^2 sigma^2 per window (interior), so
    # SSIM = (2 mx my + 0.0001)/(mx^2 + my^2 + 0.0001) * (2 a s^2 + 0.0009)/((1 + a^2) s^2 + 0.0009)
    rng = np.random.default_rng(3)
    x = rng.random((36, 36))
    mx, s2 = _scipy_moments(x)
    inner = (slice(5, -5), slice(5, -5))
    for a, b in ((0.5, 0.2), (1.0, 0.0), (-1.0, 1.0), (2.0, -0.3)):
        y = a * x + b
        my = a * mx + b
        want = ((2 * mx * my + 0.0001) / (mx * mx + my * my + 0.0001)) * \
               ((2 * a * s2 + 0.0009) / ((1 + a * a) * s2 + 0.0009))
        np.testing.assert_allclose(oas.ssim_map(x, y)[inner], want[inner], rtol=1e-9, atol=1e-12)


def test_ssim_anticorrelated_pair_separates_covariance_from_product_of_deviations():
    # y = 1 - x: sigma_xy = -sigma^2 while sigma_x sigma_y = +sigma^2, so the structure
    # term is (0.0009 - 2 s^2) / (2 s^2 + 0.0009) < 0 where the variance is large
    rng = np.random.default_rng(4)
    x = rng.random((36, 36))
    y = 1.0 - x
    mx, s2 = _scipy_moments(x)
    inner = (slice(5, -5), slice(5, -5))
    my = 1.0 - mx
    lum = (2 * mx * my + 0.0001) / (mx * mx + my * my + 0.0001)
    cs = (0.0009 - 2 * s2) / (2 * s2 + 0.0009)
    m = oas.ssim_map(x, y)
    np.testing.assert_allclose(m[inner], (lum * cs)[inner], rtol=1e-9, atol=1e-12)
    assert (m[inner] < 0).all()
    assert oas.ssim(np.stack([x] * 3), np.stack([y] * 3)) < 0
