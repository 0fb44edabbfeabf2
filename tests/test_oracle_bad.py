"""Pins for the oracle's BAD descriptor (Sec. III-A: decision stump on the
difference of two box averages, computed from the integral image).

Each pin fixes the expected bits independently of the oracle: direct pixel
sums with numpy slicing, the ORB special case (5x5 box filter, theta = 0)
through scipy's uniform filter, closed forms on constant and ramp images,
symmetries (complement, translation, quarter-turn) and the exact threshold
comparison at a value where float32 rounding of the feature would decide
wrongly."""
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_2108_08380_amd import synth


def kp_array(rows):
    kp = np.zeros(len(rows), dtype=synth.KEYPOINT_DTYPE)
    for i, (x, y, s, a) in enumerate(rows):
        kp[i] = (x, y, s, a)
    return kp


def pair_array(rows):
    p = np.zeros(len(rows), dtype=synth.BOX_PAIR_DTYPE)
    for i, (x1, y1, x2, y2, r, th) in enumerate(rows):
        p[i]["x1"], p[i]["y1"], p[i]["x2"], p[i]["y2"] = x1, y1, x2, y2
        p[i]["radius"], p[i]["threshold"] = r, th
    return p


def unpack(codes, n_bits):
    return np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")[:, :n_bits]


def describe(ref, img, kp, pairs):
    codes, ties = ref.describe_bad(ref.build_integral(img), kp, pairs)
    return unpack(codes, len(pairs)), ties


def direct_box_sum(img, cx, cy, R):
    return int(img[cy - R:cy + R + 1, cx - R:cx + R + 1].astype(np.int64).sum())


def test_brute_force_box_sums_axis_aligned(ref):
    """Integer keypoint, angle 0, integer scale: centres are kp + scale*u exactly.
    The bit must equal [S1 - S2 <= theta * A] with S from direct pixel sums."""
    rng = np.random.default_rng(10)
    img = rng.integers(0, 256, (120, 140), dtype=np.uint8)
    pairs = synth.box_pairs(rng, 256, max_offset=14, radius_range=(0, 5), threshold_range=(-30, 30))
    kps = kp_array([(70, 60, 1.0, 0.0), (65, 58, 2.0, 0.0), (71, 61, 3.0, 0.0)])
    bits, ties = describe(ref, img, kps, pairs)
    assert ties == 0
    for i, kp in enumerate(kps):
        s = int(kp["scale"])
        for j, p in enumerate(pairs):
            R = int(p["radius"]) * s
            c1 = (int(kp["x"]) + s * int(p["x1"]), int(kp["y"]) + s * int(p["y1"]))
            c2 = (int(kp["x"]) + s * int(p["x2"]), int(kp["y"]) + s * int(p["y2"]))
            d = direct_box_sum(img, *c1, R) - direct_box_sum(img, *c2, R)
            assert bits[i, j] == int(d <= float(p["threshold"]) * (2 * R + 1) ** 2), (i, j)


def test_orb_special_case_5x5_box_filter(ref):
    """ORB's features are BAD features with a 5x5 box and theta = 0 (Sec. IV-A
    ablation): bit = [mean5(c1) <= mean5(c2)], mean5 from scipy's uniform filter."""
    rng = np.random.default_rng(11)
    img = rng.integers(0, 256, (90, 100), dtype=np.uint8)
    mean5 = ndimage.uniform_filter(img.astype(np.float64), size=5, mode="constant")
    pairs = synth.box_pairs(rng, 512, max_offset=14, radius_range=(2, 2), threshold_range=(0, 0))
    kps = kp_array([(50, 45, 1.0, 0.0), (40, 41, 1.0, 0.0)])
    bits, _ = describe(ref, img, kps, pairs)
    for i, kp in enumerate(kps):
        for j, p in enumerate(pairs):
            a = mean5[int(kp["y"]) + p["y1"], int(kp["x"]) + p["x1"]]
            b = mean5[int(kp["y"]) + p["y2"], int(kp["x"]) + p["x2"]]
            # means are k/25 for integers k: compare the integer sums to avoid rounding
            assert bits[i, j] == int(round(a * 25) <= round(b * 25)), (i, j)


def test_constant_image_gives_threshold_sign(ref):
    img = np.full((80, 80), 93, dtype=np.uint8)
    rng = np.random.default_rng(12)
    pairs = synth.box_pairs(rng, 256, threshold_range=(-3, 3))
    kps = synth.keypoints(rng, 20, 80, 80, border=20)
    bits, _ = describe(ref, img, kps, pairs)
    expect = (pairs["threshold"] >= 0).astype(np.uint8)
    assert (bits == expect[None, :]).all()


def test_bit_packing_order(ref):
    """Bit j lives in word j // 64 at position j % 64 (LSB first)."""
    img = np.zeros((64, 64), dtype=np.uint8)
    for j in [0, 1, 63, 64, 100, 255]:
        th = np.full(256, -1.0, dtype=np.float32)
        th[j] = 0.0
        pairs = pair_array([(0, 0, 0, 0, 1, float(v)) for v in th])
        codes, _ = ref.describe_bad(ref.build_integral(img), kp_array([(32, 32, 1.0, 0.0)]), pairs)
        expect = np.zeros(4, dtype=np.uint64)
        expect[j // 64] = np.uint64(1) << np.uint64(j % 64)
        np.testing.assert_array_equal(codes[0], expect)


def test_integer_ramp_closed_form(ref):
    """I(x, y) = x: a box mean equals its centre column, so bit = [c1x - c2x <= theta]."""
    W, H = 200, 120
    img = np.tile(np.arange(W, dtype=np.uint8), (H, 1))
    rng = np.random.default_rng(13)
    pairs = synth.box_pairs(rng, 256, threshold_range=(-20, 20))
    kps = kp_array([(100, 60, 1.0, 0.0), (90, 55, 2.0, 0.0)])
    bits, _ = describe(ref, img, kps, pairs)
    for i, kp in enumerate(kps):
        s = int(kp["scale"])
        expect = ((s * pairs["x1"].astype(int) - s * pairs["x2"].astype(int)) <= pairs["threshold"]).astype(np.uint8)
        np.testing.assert_array_equal(bits[i], expect)


def test_complement_negates_feature(ref):
    """255 - I negates every feature: [-f <= 0] = 1 - [f < 0].  A sign slip in
    f (S2 - S1 instead of S1 - S2) still passes this, so the ramp pin above
    carries the sign; this one carries the strict/non-strict comparison."""
    rng = np.random.default_rng(14)
    img = synth.quantize_u8(synth.grey_image(rng, 160, 120, n_rect=10))
    pairs = synth.box_pairs(rng, 512, threshold_range=(0, 0))
    kps = synth.keypoints(rng, 50, 160, 120, border=40, scale_range=(1.0, 1.5))
    b_comp, _ = describe(ref, 255 - img, kps, pairs)
    strict = pairs.copy()
    # box areas are at most 17^2 here, so f <= -1e-4 holds exactly when S1 - S2 <= -1
    strict["threshold"] = -1e-4
    lt, _ = describe(ref, img, kps, strict)
    np.testing.assert_array_equal(b_comp, 1 - lt)
    assert 0 < lt.mean() < 1


def test_integer_translation_invariance(ref):
    """Moving the scene and the keypoints by the same integer offset leaves the
    codes unchanged while no box touches the border."""
    rng = np.random.default_rng(15)
    big = synth.quantize_u8(synth.grey_image(rng, 300, 240, n_rect=20))
    pairs = synth.box_pairs(rng, 256)
    kps = synth.keypoints(rng, 40, 200, 200, border=80, scale_range=(1.0, 1.6))
    kps["x"] = np.round(kps["x"] * 1024) / 1024  # exact in float32 after the shift
    kps["y"] = np.round(kps["y"] * 1024) / 1024
    a, ta = describe(ref, big[21:221, 37:237], kps, pairs)
    b, tb = describe(ref, big, synth.shift_keypoints(kps, 37, 21), pairs)
    assert ta == 0 and tb == 0
    np.testing.assert_array_equal(a, b)


def test_quarter_turn_equals_rotated_offsets(ref):
    """angle = pi/2 maps offset (ux, uy) to (-uy, ux): the descriptor equals the
    angle-0 descriptor of the rotated pair table.  Keypoints sit at .25 so the
    tiny cos(pi/2) residue never crosses a rounding tie."""
    rng = np.random.default_rng(16)
    img = synth.quantize_u8(synth.grey_image(rng, 200, 200, n_rect=20))
    pairs = synth.box_pairs(rng, 256)
    rot = pairs.copy()
    rot["x1"], rot["y1"] = -pairs["y1"], pairs["x1"]
    rot["x2"], rot["y2"] = -pairs["y2"], pairs["x2"]
    for s in (1.0, 2.0, 3.0):
        kp90 = kp_array([(100.25, 99.25, s, math.pi / 2)])
        kp0 = kp_array([(100.25, 99.25, s, 0.0)])
        a, ta = describe(ref, img, kp90, pairs)
        b, tb = describe(ref, img, kp0, rot)
        assert ta == 0 and tb == 0
        np.testing.assert_array_equal(a, b)


def test_exact_threshold_comparison(ref):
    """f <= theta is decided exactly (S1 - S2 <= theta * A), not on a float32 feature."""
    # find d, A (A = 9: radius 1) with float32(d / A) < d / A
    A = 9
    d = next(d for d in range(1, 200) if float(np.float32(d / A)) < d / A)
    theta = float(np.float32(d / A))  # slightly below the true feature d/A
    img = np.zeros((40, 40), dtype=np.uint8)
    img[20, 20] = d  # box at u1 = (0, 0) around (20, 20) sums to d, box at u2 is all zero
    pairs = pair_array([(0, 0, 10, 0, 1, theta), (0, 0, 10, 0, 1, float(np.nextafter(np.float32(d / A), np.float32(np.inf))))]
                       + [(0, 0, 10, 0, 1, -100.0)] * 62)
    bits, _ = describe(ref, img, kp_array([(20, 20, 1.0, 0.0)]), pairs)
    assert bits[0, 0] == 0  # d/A > theta although float32(d/A) == theta
    assert bits[0, 1] == 1


def test_border_clamp(ref):
    """Box centres are clamped so the whole box of radius R lies in the image."""
    rng = np.random.default_rng(17)
    img = rng.integers(0, 256, (50, 60), dtype=np.uint8)
    pairs = pair_array([(-14, -14, 14, 14, 3, 0.0)] + [(14, -14, -14, 14, 2, 5.0)] * 63)
    kps = kp_array([(2, 3, 1.0, 0.0), (57, 47, 1.0, 0.0)])
    bits, _ = describe(ref, img, kps, pairs)
    for i, kp in enumerate(kps):
        for j, p in enumerate(pairs[:2]):
            R = int(p["radius"])
            c = [int(np.clip(kp["x"] + p["x1"], R, 59 - R)), int(np.clip(kp["y"] + p["y1"], R, 49 - R)),
                 int(np.clip(kp["x"] + p["x2"], R, 59 - R)), int(np.clip(kp["y"] + p["y2"], R, 49 - R))]
            dd = direct_box_sum(img, c[0], c[1], R) - direct_box_sum(img, c[2], c[3], R)
            assert bits[i, j] == int(dd <= float(p["threshold"]) * (2 * R + 1) ** 2)


def test_radius_cap_small_image(ref):
    """Scaled radii larger than the image allows are capped at (min(W, H) - 1) / 2."""
    img = np.arange(7 * 9, dtype=np.uint8).reshape(7, 9)
    pairs = pair_array([(0, 0, 0, 0, 5, 0.0)] * 64)
    bits, _ = describe(ref, img, kp_array([(4, 3, 4.0, 0.3)]), pairs)
    assert bits.all()  # identical boxes: f = 0 <= 0


def test_invalid_keypoints_zero_code(ref):
    img = np.full((64, 64), 10, dtype=np.uint8)
    pairs = pair_array([(0, 0, 0, 0, 1, 0.0)] * 64)
    kps = kp_array([(np.nan, 30, 1, 0), (30, np.inf, 1, 0), (30, 30, 0.0, 0), (30, 30, -1.0, 0),
                    (30, 30, 1.0, np.nan), (30, 30, 1.0, 0.0)])
    bits, _ = describe(ref, img, kps, pairs)
    assert not bits[:5].any() and bits[5].all()


@pytest.mark.parametrize("seed_offset", [0])
def test_config_workload_has_no_near_ties(ref, seed_offset):
    w = synth.bad256_pair(synth.SEED_BASE + seed_offset)
    for img, kp in ((w.image1, w.kp1), (w.image2, w.kp2)):
        _, ties = ref.describe_bad(ref.build_integral(img), kp, w.pairs)
        assert ties == 0


def _exact_centre_half_up(k, s, u):
    """Nearest pixel to k + s*u with halves rounded up, in exact rationals
    (k and s are float32 values, u an integer offset)."""
    from fractions import Fraction
    return math.floor(Fraction(float(k)) + Fraction(float(s)) * u + Fraction(1, 2))


def _exact_radius_half_up(r, s):
    from fractions import Fraction
    return math.floor(Fraction(int(r)) * Fraction(float(s)) + Fraction(1, 2))


@pytest.mark.parametrize("scale", [1.5, 2.5, 3.5, 3.49])
def test_fractional_scale_radius_rounds_to_nearest(ref, scale):
    """Sec. III-A gives both boxes one size s; the scaled radius r*scale is
    rounded to the nearest integer (halves up).  At these scales r*scale has a
    fractional part >= 0.5 for some r, so truncation would give a smaller box.
    Expected bits come from direct pixel sums over boxes whose radius and
    centres are computed in exact rationals."""
    rng = np.random.default_rng(100 + int(scale * 100))
    img = rng.integers(0, 256, (220, 240), dtype=np.uint8)
    pairs = synth.box_pairs(rng, 256, max_offset=14, radius_range=(1, 5), threshold_range=(-30, 30))
    s32 = np.float32(scale)
    # a .25 offset keeps every centre of the half-integer scales off a rounding tie
    kps = kp_array([(120.25, 110.25, s32, 0.0), (118.25, 107.75, s32, 0.0)])
    bits, ties = describe(ref, img, kps, pairs)
    assert ties == 0
    n_round_up = 0
    for i, kp in enumerate(kps):
        for j, p in enumerate(pairs):
            R = _exact_radius_half_up(p["radius"], s32)
            n_round_up += R != math.floor(float(p["radius"]) * float(s32))
            c1 = (_exact_centre_half_up(kp["x"], s32, int(p["x1"])), _exact_centre_half_up(kp["y"], s32, int(p["y1"])))
            c2 = (_exact_centre_half_up(kp["x"], s32, int(p["x2"])), _exact_centre_half_up(kp["y"], s32, int(p["y2"])))
            d = direct_box_sum(img, *c1, R) - direct_box_sum(img, *c2, R)
            assert bits[i, j] == int(d <= float(p["threshold"]) * (2 * R + 1) ** 2), (i, j, R)
    assert n_round_up > 0  # the pin exercises radii that truncation would shrink


@pytest.mark.parametrize("scale", [1.0, 2.0, 3.0])
def test_half_pixel_centres_round_up(ref, scale):
    """A keypoint on a half-pixel position with angle 0 and integer scale puts
    every box centre exactly halfway between two pixels; the centre is the
    pixel above (x + 1/2 -> x + 1), on both axes and for even and odd pixels.
    Expected bits from direct pixel sums at those centres."""
    rng = np.random.default_rng(200 + int(scale))
    img = rng.integers(0, 256, (200, 210), dtype=np.uint8)
    pairs = synth.box_pairs(rng, 512, max_offset=14, radius_range=(1, 5), threshold_range=(-30, 30))
    kps = kp_array([(100.5, 90.5, scale, 0.0), (101.5, 91.5, scale, 0.0), (100.5, 91.0, scale, 0.0)])
    bits, ties = describe(ref, img, kps, pairs)
    assert ties == 0
    s = int(scale)
    for i, kp in enumerate(kps):
        xf, yf = math.floor(float(kp["x"])), math.floor(float(kp["y"]))
        up_x = 1 if float(kp["x"]) != xf else 0
        up_y = 1 if float(kp["y"]) != yf else 0
        for j, p in enumerate(pairs):
            R = int(p["radius"]) * s
            c1 = (xf + s * int(p["x1"]) + up_x, yf + s * int(p["y1"]) + up_y)
            c2 = (xf + s * int(p["x2"]) + up_x, yf + s * int(p["y2"]) + up_y)
            d = direct_box_sum(img, *c1, R) - direct_box_sum(img, *c2, R)
            assert bits[i, j] == int(d <= float(p["threshold"]) * (2 * R + 1) ** 2), (i, j)
