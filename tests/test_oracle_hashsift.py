"""Pins for the oracle's HashSIFT descriptor (Sec. III-B: SIFT features of the
normalized 32x32 patch, binarized as sgn(B [f; 1])).

With scale 1, angle 0 and a keypoint at (x0 + 15.5, y0 + 15.5) every patch
sample falls on a pixel centre, so the patch equals an image crop exactly and
the histogram of ramp and parabola images has a closed form: a product of
one-dimensional sums of the Gaussian window against the triangular cell
weights, with all gradient mass in known orientation bins.  The parabola is
not symmetric in x and y, so it also fixes the (cy, cx, o) layout."""
import math

import numpy as np
import pytest

from paper_2108_08380_amd import synth


def kp_array(rows):
    kp = np.zeros(len(rows), dtype=synth.KEYPOINT_DTYPE)
    for i, r in enumerate(rows):
        kp[i] = r
    return kp


J = np.arange(32)
GAUSS = np.exp(-((J - 15.5) ** 2) / (2 * 16.0**2))


def tri(c):
    """Triangular weight of patch column/row j for spatial cell c (centres 8c + 3.5)."""
    return np.maximum(0.0, 1.0 - np.abs((J + 0.5) / 8.0 - 0.5 - c))


CELL = np.array([np.sum(GAUSS * tri(c)) for c in range(4)])


def closed_form(cy_profile, cx_profile_by_bin):
    """h[cy, cx, o] = cy_profile[cy] * cx_profile_by_bin[o][cx], then L2-normalized."""
    h = np.zeros((4, 4, 8))
    for o, prof in cx_profile_by_bin.items():
        h[:, :, o] = np.outer(cy_profile, prof)
    h = h.reshape(-1)
    return h / np.linalg.norm(h)


def aligned_patch_image(fn, size=64):
    """f32 image I[y, x] = fn(x, y) and the keypoint whose patch is its centre crop."""
    y, x = np.mgrid[0:size, 0:size].astype(np.float64)
    img = fn(x, y).astype(np.float32)
    assert np.array_equal(img.astype(np.float64), fn(x, y)), "values must be exact in float32"
    c = size / 2 - 0.5
    return img, kp_array([(c, c, 1.0, 0.0)])


@pytest.mark.parametrize("sign,bin_", [(1, 0), (-1, 4)])
def test_x_ramp_closed_form(ref, sign, bin_):
    img, kp = aligned_patch_image(lambda x, y: 0.5 + sign * x / 256.0)
    f = ref.hashsift_hist(img, kp)[0]
    np.testing.assert_allclose(f, closed_form(CELL, {bin_: CELL}), atol=1e-12)


@pytest.mark.parametrize("sign,bin_", [(1, 2), (-1, 6)])
def test_y_ramp_closed_form(ref, sign, bin_):
    img, kp = aligned_patch_image(lambda x, y: 0.5 + sign * y / 256.0)
    f = ref.hashsift_hist(img, kp)[0]
    np.testing.assert_allclose(f, closed_form(CELL, {bin_: CELL}), atol=1e-12)


def test_diagonal_ramp_closed_form(ref):
    img, kp = aligned_patch_image(lambda x, y: (x + y) / 256.0)
    f = ref.hashsift_hist(img, kp)[0]
    np.testing.assert_allclose(f, closed_form(CELL, {1: CELL}), atol=1e-12)


def test_oblique_ramp_splits_between_two_bins(ref):
    beta = 0.3  # gradient direction; bin coordinate 0.3 * 8 / (2 pi) = 0.382
    ramp = lambda x, y: np.float32((math.cos(beta) * x + math.sin(beta) * y) / 256.0).astype(np.float64)
    img, kp = aligned_patch_image(ramp)
    f = ref.hashsift_hist(img, kp)[0]
    bo = beta * 8 / (2 * math.pi)
    expect = closed_form(CELL, {0: (1 - bo) * CELL, 1: bo * CELL})
    # the float32 image rounds the ramp: gradients are constant to ~1e-7 relative
    np.testing.assert_allclose(f, expect, atol=2e-5)


def test_parabola_fixes_spatial_layout(ref):
    """I = a (x - xc)^2: gx = 4a (j - 15.5), gy = 0.  Columns right of the centre
    vote into bin 0, columns left of it into bin 4, with weight |j - 15.5|."""
    a = 2.0**-10
    img, kp = aligned_patch_image(lambda x, y: a * (x - 31.5) ** 2)
    f = ref.hashsift_hist(img, kp)[0]
    mag = 4 * a * np.abs(J - 15.5)
    right = np.array([np.sum(mag * GAUSS * tri(c) * (J > 15.5)) for c in range(4)])
    left = np.array([np.sum(mag * GAUSS * tri(c) * (J < 15.5)) for c in range(4)])
    np.testing.assert_allclose(f, closed_form(CELL, {0: right, 4: left}), atol=1e-12)
    # the transposed parabola puts the same profile along y, in bins 2 and 6
    imgT, kpT = aligned_patch_image(lambda x, y: a * (y - 31.5) ** 2)
    fT = ref.hashsift_hist(imgT, kpT)[0].reshape(4, 4, 8)
    hT = np.zeros((4, 4, 8))
    hT[:, :, 2] = np.outer(right, CELL)
    hT[:, :, 6] = np.outer(left, CELL)
    np.testing.assert_allclose(fT.reshape(-1), hT.reshape(-1) / np.linalg.norm(hT), atol=1e-12)
    assert not np.allclose(f, fT.reshape(-1), atol=1e-3)


@pytest.mark.parametrize("dtype", [np.uint8, np.float32])
def test_constant_image_gives_zero_histogram(ref, dtype):
    img = np.full((80, 90), 77 if dtype == np.uint8 else 0.3, dtype=dtype)
    rng = np.random.default_rng(20)
    kps = synth.keypoints(rng, 16, 90, 80, border=10, scale_range=(0.5, 6))
    B, t = synth.projection(rng, 256)
    hist, resp, codes = ref.describe_hashsift(img, kps, B, t)
    assert not hist.any()
    np.testing.assert_array_equal(resp, -np.broadcast_to(t.astype(np.float64), resp.shape))
    bits = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")
    np.testing.assert_array_equal(bits, np.broadcast_to((t < 0).astype(np.uint8), bits.shape))


def test_quarter_turn_of_the_image(ref):
    """Rotating the image a quarter turn and the keypoint frame with it leaves the
    features unchanged: np.rot90 maps (x, y) to (y, W - 1 - x) and angles to a - pi/2."""
    rng = np.random.default_rng(21)
    W, H = 160, 120
    img = (synth.value_noise(rng, H, W) / 255.0).astype(np.float32)
    kps = synth.keypoints(rng, 12, W, H, border=45, scale_range=(1.0, 1.8))
    rot = np.ascontiguousarray(np.rot90(img))
    kr = kps.copy()
    kr["x"], kr["y"] = kps["y"], (W - 1) - kps["x"]
    kr["angle"] = kps["angle"] - np.float32(math.pi / 2)
    f1 = ref.hashsift_hist(img, kps)
    f2 = ref.hashsift_hist(rot, kr)
    np.testing.assert_allclose(f1, f2, atol=1e-4)
    assert np.abs(f1).max() > 0.1


def test_normalization_and_invariances(ref):
    rng = np.random.default_rng(22)
    img = (synth.grey_image(rng, 120, 100, n_rect=8) / 255.0).astype(np.float32)
    kps = synth.keypoints(rng, 20, 120, 100, border=30, scale_range=(1.0, 2.0))
    f = ref.hashsift_hist(img, kps)
    np.testing.assert_allclose(np.linalg.norm(f, axis=1), 1.0, atol=1e-12)
    assert (f >= 0).all()
    np.testing.assert_array_equal(ref.hashsift_hist(img * np.float32(2), kps), f)  # exact power-of-2 scaling
    # the float32 offset image rounds each pixel by up to 3e-8
    np.testing.assert_allclose(ref.hashsift_hist(img + np.float32(0.25), kps), f, atol=1e-6)


def test_u8_matches_f32_rendering(ref):
    rng = np.random.default_rng(23)
    u8 = synth.quantize_u8(synth.grey_image(rng, 100, 90, n_rect=6))
    kps = synth.keypoints(rng, 10, 100, 90, border=20, scale_range=(1.0, 3.0))
    f8 = ref.hashsift_hist(u8, kps)
    f32 = ref.hashsift_hist((u8 / 255.0).astype(np.float32), kps)
    np.testing.assert_allclose(f8, f32, atol=1e-6)


def test_projection_matches_numpy(ref):
    rng = np.random.default_rng(24)
    hist = rng.random((37, 128))
    hist /= np.linalg.norm(hist, axis=1, keepdims=True)
    for n_bits in (256, 512):
        B, t = synth.projection(rng, n_bits)
        resp, codes = ref.hashsift_project(hist, B, t)
        expect = hist @ B.astype(np.float64).T - t.astype(np.float64)
        np.testing.assert_allclose(resp, expect, atol=1e-13)
        bits = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")
        np.testing.assert_array_equal(bits, (expect > 0).astype(np.uint8))


def test_invalid_keypoints(ref):
    rng = np.random.default_rng(25)
    img = rng.random((60, 60)).astype(np.float32)
    kps = kp_array([(np.nan, 30, 1, 0), (30, 30, 0, 0), (30, 30, 1, np.inf), (30, 30, 1.5, 0.4)])
    B, t = synth.projection(rng, 256)
    t[:] = -np.abs(t)  # every valid bit with f = 0 would be set
    hist, resp, codes = ref.describe_hashsift(img, kps, B, t)
    assert not hist[:3].any() and hist[3].any()
    assert not codes[:3].any() and codes[3].any()


def test_border_samples_clamp_to_edge(ref):
    """A keypoint on the image corner samples clamp-to-edge: equal to the same
    keypoint in the image padded by edge replication."""
    rng = np.random.default_rng(26)
    img = rng.random((40, 50)).astype(np.float32)
    kps = kp_array([(0.25, 1.75, 1.2, 0.7), (49.0, 39.0, 0.8, 2.0)])  # exact after the shift
    pad = 30
    big = np.pad(img, pad, mode="edge")
    kb = kps.copy()
    kb["x"] += pad
    kb["y"] += pad
    np.testing.assert_allclose(ref.hashsift_hist(img, kps), ref.hashsift_hist(big, kb), atol=1e-12)
