"""BAD codes on the GPU against the oracle, bit for bit."""
import math

import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu


def run_both(ref, dev, img, kps, pairs, n_bits=None):
    ii_np = ref.build_integral(img)
    exp, ties = ref.describe_bad(ii_np, kps, pairs, n_bits)
    ii = bd.build_integral(torch.from_numpy(img).to(dev))
    got = to_np(bd.describe_bad(ii, bd.keypoints_tensor(kps, dev), bd.pairs_tensor(pairs, dev), n_bits))
    return got, exp, ties


@pytest.mark.parametrize("n_bits", [256, 512])
def test_config_workload_bit_exact(ref, dev, n_bits):
    """640x480, 1000 keypoints, scale U[1,4], both views of the scene."""
    w = synth.bad256_pair(n_bits=n_bits)
    for img, kp in ((w.image1, w.kp1), (w.image2, w.kp2)):
        got, exp, ties = run_both(ref, dev, img, kp, w.pairs)
        assert ties == 0
        np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("n_kp", [1, 3, 4, 5, 63, 65, 257])
def test_ragged_keypoint_counts(ref, dev, n_kp):
    rng = np.random.default_rng(100 + n_kp)
    img = synth.quantize_u8(synth.grey_image(rng, 333, 211, n_rect=20))
    kps = synth.keypoints(rng, n_kp, 333, 211, border=0.0, scale_range=(0.3, 6.0))
    pairs = synth.box_pairs(rng, 256)
    got, exp, ties = run_both(ref, dev, img, kps, pairs)
    assert ties == 0
    np.testing.assert_array_equal(got, exp)


def test_border_clamp_and_radius_cap(ref, dev):
    """Keypoints on and beyond the border, scales whose boxes exceed a small image."""
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, (23, 31), dtype=np.uint8)
    kps = np.zeros(8, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(0, 0, 1, 0), (30, 22, 2, 1), (-5, 40, 1, 2), (15, 11, 9, 0.5), (15.5, 11.5, 0.2, 3),
              (1e6, -1e6, 1, 0), (12, 12, 1000.0, 4.0), (3.5, 19.5, 1.5, 0.0)]
    pairs = synth.box_pairs(rng, 512)
    got, exp, _ = run_both(ref, dev, img, kps, pairs)
    np.testing.assert_array_equal(got, exp)


def test_invalid_keypoints_give_zero_codes(ref, dev):
    img = np.full((64, 64), 90, dtype=np.uint8)
    kps = np.zeros(6, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(np.nan, 3, 1, 0), (3, np.inf, 1, 0), (3, 3, 0, 0), (3, 3, -2, 0), (3, 3, 1, np.nan), (30, 30, 1, 0)]
    pairs = synth.box_pairs(np.random.default_rng(8), 256, threshold_range=(0, 0))
    got, exp, _ = run_both(ref, dev, img, kps, pairs)
    np.testing.assert_array_equal(got, exp)
    assert not got[:5].any() and (got[5] == np.uint64(2**64 - 1)).all()


def test_exact_ties_round_half_up(ref, dev):
    """Half-integer box centres (angle 0, integer scale) round up on both sides."""
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, (100, 100), dtype=np.uint8)
    kps = np.zeros(4, dtype=synth.KEYPOINT_DTYPE)
    kps[:] = [(50.5, 50.5, 1, 0), (40.5, 60, 2, 0), (60, 40.5, 3, 0), (45.5, 45.5, 1, math.pi)]
    pairs = synth.box_pairs(rng, 256)
    got, exp, _ = run_both(ref, dev, img, kps, pairs)
    np.testing.assert_array_equal(got, exp)


def test_empty_keypoint_set(dev):
    ii = bd.build_integral(torch.zeros((10, 10), dtype=torch.uint8, device=dev))
    pairs = bd.pairs_tensor(synth.box_pairs(np.random.default_rng(1), 256), dev)
    out = bd.describe_bad(ii, torch.zeros((0, 4), dtype=torch.float32, device=dev), pairs)
    assert out.shape == (0, 4)


def test_deterministic(ref, dev):
    w = synth.bad256_pair()
    ii = bd.build_integral(torch.from_numpy(w.image1).to(dev))
    kps, pairs = bd.keypoints_tensor(w.kp1, dev), bd.pairs_tensor(w.pairs, dev)
    a = to_np(bd.describe_bad(ii, kps, pairs))
    b = to_np(bd.describe_bad(ii, kps, pairs))
    np.testing.assert_array_equal(a, b)


def test_large_image_many_keypoints(ref, dev):
    """Largest image of the batched workload (4000 x 3000) with 20000 keypoints, BAD-512."""
    rng = np.random.default_rng(11)
    img = synth.quantize_u8(synth.grey_image(rng, 4000, 3000))
    kps = synth.keypoints(rng, 20000, 4000, 3000)
    pairs = synth.box_pairs(rng, 512)
    got, exp, ties = run_both(ref, dev, img, kps, pairs)
    assert ties == 0
    np.testing.assert_array_equal(got, exp)


def test_keypoint_order_is_a_permutation(dev):
    for (W, H, n) in [(640, 480, 1000), (1920, 1080, 5000), (4000, 3000, 20000), (50, 30, 7), (64, 64, 1)]:
        kps = synth.keypoints(np.random.default_rng(n), n, W, H, border=0.0)
        order = to_np(bd.keypoint_order(bd.keypoints_tensor(kps, dev), W, H))
        np.testing.assert_array_equal(np.sort(order), np.arange(n))


def test_keypoint_order_groups_cells(dev):
    """Consecutive entries of the order are spatial neighbours: the mean step
    between consecutive keypoints is far below that of the input order."""
    W, H, n = 1920, 1080, 5000
    kps = synth.keypoints(np.random.default_rng(1), n, W, H)
    order = to_np(bd.keypoint_order(bd.keypoints_tensor(kps, dev), W, H))
    xy = np.stack([kps["x"], kps["y"]], 1)
    step = lambda p: np.linalg.norm(np.diff(p, axis=0), axis=1).mean()
    assert step(xy[order]) < 0.2 * step(xy)


def _cell_keys(kps, W, H):
    """Morton cell key of each keypoint in the 64 x 64 grid of the order, in
    float32 as the device forms it (cell side ceil(max(W, H) / 64))."""
    inv = np.float32(1.0) / np.float32(max((max(W, H) + 63) // 64, 1))

    def cell(v):
        f = v.astype(np.float32) * inv
        return np.where(f >= 64, 63, np.where(f >= 0, np.floor(f), 0)).astype(np.uint32)

    def spread(v):
        out = np.zeros_like(v)
        for b in range(6):
            out |= ((v >> b) & 1) << (2 * b)
        return out

    return spread(cell(kps["x"])) | (spread(cell(kps["y"])) << 1)


@pytest.mark.parametrize("W,H,n", [(1920, 1080, 5000), (1920, 1080, 12000), (640, 480, 1000), (37, 29, 40),
                                   (4000, 3000, 20000), (300, 200, 1), (300, 200, 0)])
def test_integral_and_order_in_one_call(dev, W, H, n):
    """bd_build_integral_order: the integral image equals bd_build_integral's
    bit for bit, and the order is a permutation whose cell keys never
    decrease, like bd_keypoint_order's (more than 8192 keypoints take the
    sort's second loop)."""
    rng = np.random.default_rng(W + n)
    img = torch.from_numpy(synth.quantize_u8(synth.grey_image(rng, W, H, n_rect=20))).to(dev)
    kps_np = synth.keypoints(rng, n, W, H, border=0.0)
    kps = bd.keypoints_tensor(kps_np, dev)
    ii, order = bd.build_integral_order(img, kps)
    np.testing.assert_array_equal(to_np(ii), to_np(bd.build_integral(img)))
    o_fused, o_sep = to_np(order), to_np(bd.keypoint_order(kps, W, H))
    keys = _cell_keys(kps_np, W, H)
    for o in (o_fused, o_sep):
        np.testing.assert_array_equal(np.sort(o), np.arange(n))
        assert (np.diff(keys[o].astype(np.int64)) >= 0).all()
    np.testing.assert_array_equal(keys[o_fused], keys[o_sep])


@pytest.mark.parametrize("W,H,n", [(1920, 1080, 5000), (1920, 1080, 12000), (37, 29, 40), (3, 1, 2), (1, 7, 0),
                                   (300, 2048, 100), (300, 2049, 100), (4000, 3000, 9000)])
def test_prepare_view(dev, W, H, n):
    """bd_prepare_view: the integral image equals bd_build_integral's and the
    order is bd_keypoint_order's up to ties, as for bd_build_integral_order,
    and the row-pair copy of the HashSIFT image pairs each pixel with the one
    below it (the last row with itself), bit for bit.  More than 8192
    keypoints take the sort's second loop inside the first launch; 2048 rows
    is the tallest image of the two-launch form, and 2049 or more rows go
    through the separate launches."""
    rng = np.random.default_rng(W * 3 + n)
    img = torch.from_numpy(synth.quantize_u8(synth.grey_image(rng, W, H, n_rect=20))).to(dev)
    hs = torch.from_numpy(rng.standard_normal((H, W)).astype(np.float32)).to(dev)
    kps_np = synth.keypoints(rng, n, W, H, border=0.0)
    kps = bd.keypoints_tensor(kps_np, dev)
    ii, order, rp = bd.prepare_view(img, kps, hs)
    np.testing.assert_array_equal(to_np(ii), to_np(bd.build_integral(img)))
    o = to_np(order)
    keys = _cell_keys(kps_np, W, H)
    np.testing.assert_array_equal(np.sort(o), np.arange(n))
    np.testing.assert_array_equal(keys[o], keys[to_np(bd.keypoint_order(kps, W, H))])
    h = to_np(hs)
    below = np.concatenate([h[1:], h[-1:]], axis=0)
    np.testing.assert_array_equal(to_np(rp), np.stack([h, below], axis=2))
    ii2, order2, none = bd.prepare_view(img, kps)
    assert none is None
    np.testing.assert_array_equal(to_np(ii2), to_np(ii))
    np.testing.assert_array_equal(keys[to_np(order2)], keys[o])


def test_prepare_view_padded_rows(dev):
    """bd_prepare_view and the row-pair histogram on padded rows: the
    HashSIFT image and the row-pair copy are views of wider buffers (row
    strides 1000 and 2004 floats for a 997-pixel row); the padding of the copy
    is never written and the features equal those of the float image."""
    rng = np.random.default_rng(77)
    H, W, n = 301, 997, 700
    img = torch.from_numpy(synth.quantize_u8(synth.grey_image(rng, W, H, n_rect=10))).to(dev)
    hs_full = torch.from_numpy(rng.random((H, 1000)).astype(np.float32)).to(dev)
    hs = hs_full[:, :W]
    pairs_buf = torch.full((H * 2004 + 2,), -7.0, dtype=torch.float32, device=dev)
    pairs = pairs_buf[:H * 2004].view(H, 2004)[:, :2 * W].view(H, W, 2)
    kps_np = synth.keypoints(rng, n, W, H, border=0.0)
    kps = bd.keypoints_tensor(kps_np, dev)
    ii, order, rp = bd.prepare_view(img, kps, hs, pairs=pairs)
    assert rp.data_ptr() == pairs.data_ptr()
    np.testing.assert_array_equal(to_np(ii), to_np(bd.build_integral(img)))
    h = to_np(hs)
    np.testing.assert_array_equal(to_np(rp), np.stack([h, np.concatenate([h[1:], h[-1:]], axis=0)], axis=2))
    pad = to_np(pairs_buf[:H * 2004].view(H, 2004)[:, 2 * W:])
    assert (pad == -7.0).all() and to_np(pairs_buf[H * 2004:]).tolist() == [-7.0, -7.0]
    a = to_np(bd.hashsift_features(hs, kps, order=order)).view(np.uint32)
    b = to_np(bd.hashsift_features(rp, kps, order=order)).view(np.uint32)
    np.testing.assert_array_equal(a, b)


def test_prepare_view_validation(dev):
    """The HashSIFT image and its row-pair output must come together, match
    the image's size and be float32 with 4- and 8-byte aligned rows."""
    img = torch.zeros((6, 5), dtype=torch.uint8, device=dev)
    kps = bd.keypoints_tensor(np.zeros(1, dtype=synth.KEYPOINT_DTYPE), dev)
    with pytest.raises(ValueError):
        bd.prepare_view(img, kps, torch.zeros((6, 4), dtype=torch.float32, device=dev))
    with pytest.raises(TypeError):
        bd.prepare_view(img, kps, torch.zeros((6, 5), dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        bd.prepare_view(img, kps, torch.zeros((6, 5), dtype=torch.float32, device=dev),
                        pairs=torch.zeros((6, 4, 2), dtype=torch.float32, device=dev))
    with pytest.raises(ValueError, match="both or neither"):
        bd.prepare_view(img, kps, pairs=torch.zeros((6, 5, 2), dtype=torch.float32, device=dev))


def test_ordered_describe_equals_unordered(ref, dev):
    w = synth.hashsift512_pair(n_kp=3000, n_bits=512, with_bad_bits=512)
    img = torch.from_numpy(w.extra["image1_u8"]).to(dev)
    kps = bd.keypoints_tensor(w.kp1, dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    ii = bd.build_integral(img)
    order = bd.keypoint_order(kps, img.shape[1], img.shape[0])
    a = to_np(bd.describe_bad(ii, kps, pairs))
    b = to_np(bd.describe_bad(ii, kps, pairs, order=order))
    np.testing.assert_array_equal(a, b)
    exp, _ = ref.describe_bad(to_np(ii), w.kp1, w.pairs)
    np.testing.assert_array_equal(b, exp)


def test_order_entries_out_of_range_are_skipped(dev):
    """An order with invalid entries neither faults nor touches other codes:
    keypoints it names are described, the rest keep their prior contents."""
    w = synth.bad256_pair()
    img = torch.from_numpy(w.image1).to(dev)
    kps = bd.keypoints_tensor(w.kp1, dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    ii = bd.build_integral(img)
    n = len(w.kp1)
    good = to_np(bd.describe_bad(ii, kps, pairs))
    bad_order = np.arange(n, dtype=np.int32)
    bad_order[::3] = -1
    bad_order[1::7] = n + 5
    out = torch.zeros((n, 4), dtype=torch.uint64, device=dev)
    bd.describe_bad(ii, kps, pairs, out=out, order=torch.from_numpy(bad_order).to(dev))
    got = to_np(out)
    named = np.zeros(n, bool)
    named[bad_order[(bad_order >= 0) & (bad_order < n)]] = True
    np.testing.assert_array_equal(got[named], good[named])
    assert not got[~named].any()


# ---------------------------------------------------------------- compiled tables


def compiled_vs_direct(dev, img, kp, pairs, order=True):
    ii = bd.build_integral(img)
    pt = bd.pairs_tensor(pairs, dev)
    o = bd.keypoint_order(kp, img.shape[1], img.shape[0]) if order else None
    direct = bd.describe_bad(ii, kp, pt, order=o)
    table = bd.BadTable(pt)
    compiled = bd.describe_bad(ii, kp, order=o, table=table)
    np.testing.assert_array_equal(to_np(compiled), to_np(direct))
    table.close()
    return to_np(direct)


@pytest.mark.parametrize("n_bits", [256, 512])
def test_compiled_table_equals_direct(ref, dev, n_bits):
    w = synth.hashsift512_pair(synth.SEED_BASE + 20, 1920, 1080, 3000, with_bad_bits=n_bits)
    img = torch.from_numpy(w.extra["image1_u8"]).to(dev)
    kp = w.kp1.copy()
    kp["scale"][:10] = 40.0            # boxes clamped to the image
    kp["x"][10] = np.float32(np.nan)   # invalid keypoint: zero code
    kpt = bd.keypoints_tensor(kp, dev)
    codes = compiled_vs_direct(dev, img, kpt, w.pairs)
    compiled_vs_direct(dev, img, kpt, w.pairs, order=False)
    # and the oracle on a sample
    sel = np.arange(0, 3000, 97)
    exp, _ = ref.describe_bad(ref.build_integral(w.extra["image1_u8"]), kp[sel], w.pairs)
    np.testing.assert_array_equal(codes[sel], exp)


def test_compiled_table_duplicates_and_extremes(dev):
    rng = np.random.default_rng(30)
    pairs = synth.box_pairs(rng, 512)
    pairs[1] = pairs[0]                                  # a repeated pair
    pairs[2]["x1"], pairs[2]["y1"] = pairs[3]["x2"], pairs[3]["y2"]
    pairs[2]["radius"] = pairs[3]["radius"]              # a box shared by two pairs
    pairs[4]["x1"], pairs[4]["y1"], pairs[4]["x2"], pairs[4]["y2"] = -128, 127, 127, -128
    pairs[5]["radius"] = 255
    pairs[6]["x1"] = pairs[6]["x2"]
    pairs[6]["y1"] = pairs[6]["y2"]                      # both boxes equal: f = 0
    pairs[7:64]["x1"], pairs[7:64]["y1"], pairs[7:64]["radius"] = 0, 0, 1   # many identical boxes
    img = torch.from_numpy(synth.quantize_u8(synth.grey_image(rng, 333, 251))).to(dev)
    kp = bd.keypoints_tensor(synth.keypoints(rng, 777, 333, 251, 8.0, (0.5, 6.0)), dev)
    compiled_vs_direct(dev, img, kp, pairs)
    # a tiny image where every box is clamped
    tiny = torch.from_numpy(rng.integers(0, 256, (9, 13), dtype=np.uint8)).to(dev)
    kp2 = bd.keypoints_tensor(synth.keypoints(rng, 50, 13, 9, 0.0, (1.0, 3.0)), dev)
    compiled_vs_direct(dev, tiny, kp2, pairs)
