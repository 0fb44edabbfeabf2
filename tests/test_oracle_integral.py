"""Pins for the oracle's integral image (Sec. III-A, box averages from an
integral image).  Checked against numpy's cumulative sums (an independent
library routine), brute-force rectangle sums and closed forms."""
import numpy as np
import pytest


def test_matches_numpy_cumsum(ref):
    rng = np.random.default_rng(1)
    for (h, w) in [(1, 1), (1, 9), (7, 1), (23, 37), (64, 65)]:
        img = rng.integers(0, 256, (h, w), dtype=np.uint8)
        ii = ref.build_integral(img)
        assert ii.shape == (h + 1, w + 1)
        expect = np.zeros((h + 1, w + 1), dtype=np.uint64)
        expect[1:, 1:] = img.astype(np.uint64).cumsum(0).cumsum(1)
        np.testing.assert_array_equal(ii, (expect % 2**32).astype(np.uint32))


def test_zero_border_and_total(ref):
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, (41, 53), dtype=np.uint8)
    ii = ref.build_integral(img)
    assert not ii[0].any() and not ii[:, 0].any()
    assert int(ii[-1, -1]) == int(img.astype(np.int64).sum()) % 2**32


def test_constant_image_closed_form(ref):
    c = 7
    img = np.full((30, 45), c, dtype=np.uint8)
    ii = ref.build_integral(img)
    y, x = np.mgrid[0:31, 0:46]
    np.testing.assert_array_equal(ii, (c * x * y).astype(np.uint32))


def test_rectangle_sums_brute_force(ref):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (50, 70), dtype=np.uint8)
    ii = ref.build_integral(img).astype(np.int64)
    for _ in range(300):
        y0, y1 = sorted(rng.integers(0, 51, 2))
        x0, x1 = sorted(rng.integers(0, 71, 2))
        s = (ii[y1, x1] - ii[y0, x1] - ii[y1, x0] + ii[y0, x0]) % 2**32
        assert s == int(img[y0:y1, x0:x1].astype(np.int64).sum())


def test_wraparound_keeps_box_sums_exact(ref):
    # 5000 x 4000 pixels at 255 sum to 5.1e9 > 2^32: entries wrap, box sums stay exact.
    img = np.full((4000, 5000), 255, dtype=np.uint8)
    img[::7, ::3] = 17
    ii = ref.build_integral(img)
    assert int(ii[-1, -1]) == int(img.astype(np.int64).sum()) % 2**32
    y0, y1, x0, x1 = 3500, 3541, 4900, 4941
    s = (int(ii[y1, x1]) - int(ii[y0, x1]) - int(ii[y1, x0]) + int(ii[y0, x0])) % 2**32
    assert s == int(img[y0:y1, x0:x1].astype(np.int64).sum())


@pytest.mark.parametrize("pitch_pad", [0, 3])
def test_pitch_is_respected(ref, pitch_pad):
    # The C entry point takes row strides; the wrapper passes dense ones.  A
    # padded parent array must give the same result as its dense copy.
    rng = np.random.default_rng(4)
    parent = rng.integers(0, 256, (20, 31 + pitch_pad), dtype=np.uint8)
    view = parent[:, :31]
    np.testing.assert_array_equal(ref.build_integral(view), ref.build_integral(view.copy()))
