"""HashSIFT on the GPU against the FP64 oracle.

Tolerance (FP32 kernel vs FP64 oracle), fixed here and in the design notes:
  features   |f_gpu - f_64| <= 1e-4 per element
  responses  |r_gpu - r_64| <= 1e-4 per element
  codes      every bit equal wherever |r_64| >= 2e-4 (the stated margin);
             bits inside the margin are counted and reported, not failed.
"""
import math

import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu

F_TOL = 1e-4
R_TOL = 1e-4
MARGIN = 2e-4


def unpack(codes, n_bits):
    return np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")[:, :n_bits]


def compare(ref, dev, img, kps, B, t, label=""):
    h64, r64, c64 = ref.describe_hashsift(img, kps, B, t)
    codes, hist, resp = bd.describe_hashsift(torch.from_numpy(img).to(dev), bd.keypoints_tensor(kps, dev),
                                             torch.from_numpy(B).to(dev), torch.from_numpy(t).to(dev),
                                             with_hist=True, with_resp=True)
    codes, hist, resp = to_np(codes), to_np(hist), to_np(resp)
    df = np.abs(hist - h64).max() if len(kps) else 0.0
    dr = np.abs(resp - r64).max() if len(kps) else 0.0
    n_bits = B.shape[0]
    outside = np.abs(r64) >= MARGIN
    bg, be = unpack(codes, n_bits), unpack(c64, n_bits)
    mismatch_out = int(((bg != be) & outside).sum())
    inside = int((~outside).sum())
    flips_in = int(((bg != be) & ~outside).sum())
    print(f"{label} n={len(kps)} max|df|={df:.2e} max|dr|={dr:.2e} margin responses={inside} flips inside={flips_in}")
    assert df <= F_TOL, df
    assert dr <= R_TOL, dr
    assert mismatch_out == 0
    return codes, c64


@pytest.mark.parametrize("n_bits", [256, 512])
def test_config_workload(ref, dev, n_bits):
    """1920x1080 float32 image, 5000 keypoints with scale U[1.6, 8], HashSIFT-512 (and -256)."""
    w = synth.hashsift512_pair(n_bits=n_bits)
    compare(ref, dev, w.image1, w.kp1, w.B, w.t, "view1")
    compare(ref, dev, w.image2, w.kp2, w.B, w.t, "view2")


def test_rotations_on_and_between_the_axes(ref, dev):
    """Angles on the image axes, on the diagonals and just off them, at
    small to large scales: every orientation of the 8x8 sample blocks the
    resampling walks (the block steps change sign and axis with the angle)."""
    rng = np.random.default_rng(77)
    img = (synth.grey_image(rng, 640, 480, n_rect=60) / 255.0).astype(np.float32)
    base = [k * math.pi / 4 for k in range(8)]
    angles = base + [a + d for a in base for d in (-1e-6, 1e-6)] + [-math.pi / 2, 1e-30]
    scales = [0.5, 1.6, 8.0, 20.0]
    kps = np.empty(len(angles) * len(scales), dtype=synth.KEYPOINT_DTYPE)
    i = 0
    for a in angles:
        for sc in scales:
            kps[i] = (rng.uniform(80.0, 560.0), rng.uniform(80.0, 400.0), sc, a)
            i += 1
    B, t = synth.projection(rng, 256)
    compare(ref, dev, img, kps, B, t, "rotations")


def test_u8_image(ref, dev):
    w = synth.bad256_pair()
    B, t = synth.projection(np.random.default_rng(1), 512)
    compare(ref, dev, w.image1, w.kp1, B, t, "u8")


@pytest.mark.parametrize("n_kp", [1, 3, 15, 16, 17, 63, 64, 65, 129])
def test_ragged_counts(ref, dev, n_kp):
    rng = np.random.default_rng(200 + n_kp)
    img = (synth.grey_image(rng, 300, 200, n_rect=30) / 255.0).astype(np.float32)
    kps = synth.keypoints(rng, n_kp, 300, 200, border=0.0, scale_range=(0.5, 9.0))
    B, t = synth.projection(rng, 256)
    compare(ref, dev, img, kps, B, t, f"ragged{n_kp}")


def test_flat_and_invalid_keypoints(ref, dev):
    """Patches inside a flat rectangle give f = 0 (r = -t); invalid keypoints give zero codes."""
    img = np.full((200, 200), 0.25, dtype=np.float32)
    img[:, 150:] = 0.75
    kps = np.zeros(6, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(60, 100, 1.0, 0.3), (60.3, 80.7, 1.5, 2.0), (np.nan, 5, 1, 0), (5, 5, 0.0, 0),
              (150, 100, 1.0, 0.0), (199.9, 199.9, 3.0, 1.0)]
    B, t = synth.projection(np.random.default_rng(3), 512)
    t[:] = -np.abs(t)
    codes, c64 = compare(ref, dev, img, kps, B, t, "flat")
    assert (codes[:2] == np.uint64(2**64 - 1)).all()  # f = 0, r = -t > 0 on every bit
    assert not codes[2:4].any()


def test_image_corners_clamp_to_edge(ref, dev):
    rng = np.random.default_rng(4)
    img = rng.random((37, 41)).astype(np.float32)
    kps = np.zeros(5, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(0, 0, 1, 0), (40, 36, 2, 2), (-3, 20, 1, 1), (20, 50, 0.7, 4), (20, 18, 30.0, 0.1)]
    B, t = synth.projection(rng, 256)
    compare(ref, dev, img, kps, B, t, "corners")


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("width", [1, 2, 3])
def test_narrow_images(ref, dev, width, dtype):
    """Float and u8 images 1, 2 and 3 pixels wide: the sampler reads each
    row's two pixels as one pair clamped to columns [0, W - 2] (width 1 reads
    them one by one); samples left, right and inside the columns clamp like
    the oracle."""
    rng = np.random.default_rng(20 + width)
    img = rng.random((9, width)).astype(np.float32)
    if dtype == "u8":
        img = rng.integers(0, 256, (9, width), dtype=np.uint8)
    kps = np.zeros(4, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(0, 0, 1, 0), (width - 1, 8, 0.5, 1.0), (0.5, 4, 2.0, 2.0), (width + 3.0, -2, 1.0, 3.0)]
    B, t = synth.projection(rng, 256)
    compare(ref, dev, img, kps, B, t, f"narrow-{width}")


def test_deterministic(dev):
    w = synth.hashsift512_pair(n_kp=2000)
    args = (torch.from_numpy(w.image1).to(dev), bd.keypoints_tensor(w.kp1, dev), torch.from_numpy(w.B).to(dev),
            torch.from_numpy(w.t).to(dev))
    a = bd.describe_hashsift(*args, with_hist=True, with_resp=True)
    b = bd.describe_hashsift(*args, with_hist=True, with_resp=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(to_np(x), to_np(y))


def test_codes_without_optional_outputs(dev):
    w = synth.hashsift512_pair(n_kp=700)
    args = (torch.from_numpy(w.image1).to(dev), bd.keypoints_tensor(w.kp1, dev), torch.from_numpy(w.B).to(dev),
            torch.from_numpy(w.t).to(dev))
    a = to_np(bd.describe_hashsift(*args))
    b = to_np(bd.describe_hashsift(*args, with_hist=True, with_resp=True)[0])
    np.testing.assert_array_equal(a, b)


def test_ordered_features_equal_unordered(dev):
    w = synth.hashsift512_pair(n_kp=3000)
    img = torch.from_numpy(w.image1).to(dev)
    kps = bd.keypoints_tensor(w.kp1, dev)
    order = bd.keypoint_order(kps, img.shape[1], img.shape[0])
    a = to_np(bd.hashsift_features(img, kps))
    b = to_np(bd.hashsift_features(img, kps, order=order))
    np.testing.assert_array_equal(a, b)
    B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
    c1 = to_np(bd.describe_hashsift(img, kps, B, t))
    c2 = to_np(bd.describe_hashsift(img, kps, B, t, order=order))
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(c1, to_np(bd.hashsift_project(torch.from_numpy(b).to(dev), B, t, kps)))


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_far_keypoints_and_huge_scales(ref, dev, dtype):
    """Sample positions are 32.32 fixed point while every sample of the patch
    stays within 2^30 pixels of the origin, FP64 otherwise: keypoints on both
    sides of that bound (far off the image, or with scales up to 5e7) all
    clamp to the image edges like the oracle's."""
    rng = np.random.default_rng(11)
    img = rng.random((37, 41)).astype(np.float32)
    if dtype == "u8":
        img = (img * 255).astype(np.uint8)
    kps = np.zeros(10, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(1.0e9, 20.0, 1.0, 0.5),        # fixed point, positions near 1e9
              (-1.0e9, 30.0, 2.0, 2.5),       # fixed point, negative
              (20.0, 18.0, 4.0e7, 0.2),       # fixed point, |offsets| up to 9.3e8
              (1.2e9, 20.0, 1.0, 0.5),        # FP64 path
              (20.0, -3.0e9, 3.0, 2.0),       # FP64 path
              (20.0, 18.0, 5.0e7, 0.2),       # FP64 path: scale reaches past 2^30
              (-2.0e9, -3.0e9, 3.0, 4.0),     # FP64 path, far corner
              (20.0, 18.0, 1.0e30, 1.0),      # FP64 path, absurd scale
              (40.5, 36.5, 1.0, 0.0),         # ordinary keypoints beside them
              (10.25, 30.75, 0.5, -1.0)]
    B, t = synth.projection(rng, 256)
    compare(ref, dev, img, kps, B, t, f"far-{dtype}")


def test_hashsift_image_size_limits(ref, dev):
    """Images whose row offsets do not fit the sampler's 24-bit multiplies and
    32-bit offsets are rejected before any launch; the tallest admitted image
    (2^24 - 1 rows) samples correctly at its far end."""
    B, t = synth.projection(np.random.default_rng(2), 256)
    Bd, td = torch.from_numpy(B).to(dev), torch.from_numpy(t).to(dev)
    kps = bd.keypoints_tensor(np.zeros(1, dtype=synth.KEYPOINT_DTYPE), dev)
    wide = torch.zeros((2, (1 << 24) + 64), dtype=torch.uint8, device=dev)[:, :100]  # pitch 2^24 + 64
    with pytest.raises(bd.BDError, match="2\\^24"):
        bd.describe_hashsift(wide, kps, Bd, td)
    tall = torch.zeros((1 << 24, 1), dtype=torch.uint8, device=dev)  # H = 2^24
    with pytest.raises(bd.BDError, match="2\\^24"):
        bd.hashsift_features(tall, kps)
    rng = np.random.default_rng(12)
    tall_ok = rng.integers(0, 256, size=((1 << 24) - 1, 3), dtype=np.uint8)
    kp = np.zeros(2, dtype=synth.KEYPOINT_DTYPE)
    kp[:] = [(1.0, 16777000.0, 2.0, 0.3), (1.5, 16777210.0, 1.0, 1.3)]
    compare(ref, dev, tall_ok, kp, B, t, "tall")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_empty_keypoint_set(dev, precision):
    """No keypoints: every HashSIFT call succeeds with empty outputs and the
    re-check counter is untouched."""
    rng = np.random.default_rng(7)
    img = torch.from_numpy((synth.grey_image(rng, 64, 48, n_rect=4) / 255.0).astype(np.float32)).to(dev)
    B, t = (torch.from_numpy(a).to(dev) for a in synth.projection(rng, 512))
    kps = torch.zeros((0, 4), dtype=torch.float32, device=dev)
    count = torch.zeros((1,), dtype=torch.uint32, device=dev)
    codes, hist, resp = bd.describe_hashsift(img, kps, B, t, precision=precision, with_hist=True,
                                             with_resp=True, recheck_count=count)
    assert codes.shape == (0, 8) and hist.shape == (0, 128) and resp.shape == (0, 512)
    assert bd.hashsift_features(img, kps).shape == (0, 128)
    hist0 = torch.zeros((0, 128), dtype=torch.float32, device=dev)
    assert bd.hashsift_project(hist0, B, t, precision=precision, recheck_count=count).shape == (0, 8)
    torch.cuda.synchronize()
    assert int(count.item()) == 0


def row_pairs(img):
    """Row-pair copy of a float image built with torch: (y, x) holds the
    pixel and the one below it, the last row paired with itself."""
    below = torch.cat([img[1:], img[-1:]], dim=0)
    return torch.stack([img, below], dim=2).contiguous()


def _row_pair_case(case):
    rng = np.random.default_rng(sum(case.encode()))  # stable across processes, unlike hash()
    kps = None
    if case == "workload":
        w = synth.hashsift512_pair(n_kp=3000)
        return w.image1, w.kp1
    if case.startswith("narrow"):
        width = int(case[-1])
        img = rng.random((9, width)).astype(np.float32)
        kps = np.zeros(6, dtype=synth.KEYPOINT_DTYPE)
        kps[:] = [(0, 0, 1, 0), (width - 1, 8, 0.5, 1.0), (0.5, 4, 2.0, 2.0), (width + 3.0, -2, 1.0, 3.0),
                  (-4.0, 10.5, 1.5, -2.0), (width * 0.5, 7.75, 0.25, 0.7)]
        return img, kps
    if case.startswith("short"):
        height = int(case[-1])
        img = rng.random((height, 11)).astype(np.float32)
        kps = np.zeros(5, dtype=synth.KEYPOINT_DTYPE)
        kps[:] = [(5.0, 0.0, 1.0, 0.3), (2.5, height - 0.5, 0.7, 1.9), (0.0, -3.0, 2.0, -1.0),
                  (10.0, height + 2.0, 1.5, 2.8), (7.25, 0.5, 0.4, 0.0)]
        return img, kps
    if case == "border":
        H, W = 37, 53
        img = rng.random((H, W)).astype(np.float32)
        xs = [-3.0, -0.5, 0.0, 0.25, W - 1.0, W - 0.5, W + 2.0]
        ys = [-3.0, -0.75, 0.0, 0.5, H - 1.5, H - 1.0, H - 0.25, H + 2.0]
        pts = [(x, y) for x in xs for y in ys]
        kps = np.zeros(len(pts), dtype=synth.KEYPOINT_DTYPE)
        for i, (x, y) in enumerate(pts):
            kps[i] = (x, y, rng.uniform(0.3, 3.0), rng.uniform(-math.pi, math.pi))
        return img, kps
    if case == "far":
        img = rng.random((37, 41)).astype(np.float32)
        kps = np.zeros(6, dtype=synth.KEYPOINT_DTYPE)
        kps[:] = [(1.0e9, 20.0, 1.0, 0.5), (20.0, 18.0, 4.0e7, 0.2), (1.2e9, 20.0, 1.0, 0.5),
                  (20.0, -3.0e9, 3.0, 2.0), (-2.0e9, -3.0e9, 3.0, 4.0), (40.5, 36.5, 1.0, 0.0)]
        return img, kps
    raise ValueError(case)


@pytest.mark.parametrize("case", ["workload", "narrow1", "narrow2", "narrow3", "short1", "short2", "border", "far"])
def test_row_pair_image_equals_float(ref, dev, case):
    """An (H, W, 2) row-pair image gives the float image's features,
    responses and codes bit for bit: on the 1920 x 1080 workload, on images
    1 to 3 pixels wide, on images of 1 and 2 rows, for keypoints whose
    samples fall above the first row,
    below the last or beside the columns, and on the fixed-point and FP64
    position paths.  The workload case is also held against the oracle."""
    img_np, kps_np = _row_pair_case(case)
    img = torch.from_numpy(img_np).to(dev)
    rp = row_pairs(img)
    kps = bd.keypoints_tensor(kps_np, dev)
    B, t = synth.projection(np.random.default_rng(5), 512)
    Bd, td = torch.from_numpy(B).to(dev), torch.from_numpy(t).to(dev)
    a = to_np(bd.hashsift_features(img, kps)).view(np.uint32)
    b = to_np(bd.hashsift_features(rp, kps)).view(np.uint32)
    np.testing.assert_array_equal(a, b)
    for x, y in zip(bd.describe_hashsift(img, kps, Bd, td, with_hist=True, with_resp=True),
                    bd.describe_hashsift(rp, kps, Bd, td, with_hist=True, with_resp=True)):
        np.testing.assert_array_equal(to_np(x), to_np(y))
    if case == "workload":
        compare(ref, dev, img_np, kps_np, B, t, "row-pair reference")


def test_row_pair_image_validation(dev):
    """Row-pair images must hold their pairs contiguously in float32."""
    kps = bd.keypoints_tensor(np.zeros(1, dtype=synth.KEYPOINT_DTYPE), dev)
    img = torch.zeros((8, 5), dtype=torch.float32, device=dev)
    with pytest.raises(TypeError):
        bd.hashsift_features(torch.zeros((8, 5, 2), dtype=torch.float64, device=dev), kps)
    with pytest.raises(TypeError):
        bd.hashsift_features(torch.zeros((8, 5, 3), dtype=torch.float32, device=dev), kps)
    with pytest.raises(TypeError):
        bd.hashsift_features(row_pairs(img).transpose(0, 1), kps)
    odd = torch.zeros((8 * 11 + 1,), dtype=torch.float32, device=dev)[1:].view(8, 11)[:, :10].view(8, 5, 2)
    with pytest.raises(bd.BDError, match="8-byte aligned"):
        bd.hashsift_features(odd, kps)
