"""Batched describe-and-match on the GPU (the batching extension).

Every output of a batch must equal, bit for bit, the single-image calls on
each image (integral image + BAD, HashSIFT, Hamming k-NN), whose own parity
with the oracle is established by the other GPU tests; a sample of keypoints
is also checked against the oracle directly.  Outputs must not depend on the
tuning, on graph replay or on the autotuner's choice."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth

from conftest import to_np

pytestmark = pytest.mark.gpu

# Small batch with the edge cases: an image without keypoints, a train set
# smaller than k, fewer queries than a wavefront, a tiny image (box radii
# clamped), odd widths (unaligned rows) and several tiles per image.
SMALL_SIZES = [(640, 480, 1500), (37, 29, 40), (333, 250, 0), (1025, 769, 2100), (96, 72, 1), (500, 375, 777)]


def small_workload(seed=synth.SEED_BASE + 50, sizes=SMALL_SIZES, **kw):
    return synth.batched(seed, sizes=sizes, **kw)


def upload(w, dev, hs_f32=False):
    imgs = [torch.from_numpy(np.ascontiguousarray(im)).to(dev) for im in w.images]
    hs = [(im.float() / 255.0).contiguous() for im in imgs] if hs_f32 else None
    kps = bd.keypoints_tensor(w.flat_keypoints(), dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    B = torch.from_numpy(w.B).to(dev)
    t = torch.from_numpy(w.t).to(dev)
    return imgs, hs, kps, pairs, B, t


def single_image_outputs(w, imgs, hs, kps, pairs, B, t, k=2, precision="fp32"):
    """The same work through the single-image entry points, concatenated in batch layout."""
    offs = np.concatenate([[0], np.cumsum([len(x) for x in w.kps])])
    bad, hsc = [], []
    for j, img in enumerate(imgs):
        kp = kps[offs[j]:offs[j + 1]].contiguous()
        if len(kp) == 0:
            bad.append(torch.empty((0, w.pairs.shape[0] // 64), dtype=torch.uint64, device=img.device))
            hsc.append(torch.empty((0, B.shape[0] // 64), dtype=torch.uint64, device=img.device))
            continue
        ii = bd.build_integral(img)
        bad.append(bd.describe_bad(ii, kp, pairs))
        src = hs[j] if hs is not None else img
        hsc.append(bd.describe_hashsift(src, kp, B, t, precision=precision))
    out = {"bad_codes": torch.cat(bad), "hs_codes": torch.cat(hsc)}
    for name, codes in (("bad", bad), ("hs", hsc)):
        idx, dist = [], []
        for q, tr in w.matches:
            if len(codes[q]) == 0:
                continue
            i, d = bd.match_hamming_knn(codes[q].contiguous(), codes[tr].contiguous(), k=k)
            idx.append(i)
            dist.append(d)
        out[f"{name}_idx"] = torch.cat(idx) if idx else torch.empty((0, k), dtype=torch.int32)
        out[f"{name}_dist"] = torch.cat(dist) if dist else torch.empty((0, k), dtype=torch.uint32)
    return out


def assert_same(a, b, what=""):
    assert set(a) == set(b)
    for key in a:
        x, y = to_np(a[key]), to_np(b[key])
        assert x.shape == y.shape, (what, key, x.shape, y.shape)
        np.testing.assert_array_equal(x, y, err_msg=f"{what} {key}")


def make_batch(w, imgs, hs=None, k=2, precision="fp32"):
    return bd.Batch(imgs, [len(x) for x in w.kps], w.matches, bad_bits=w.pairs.shape[0], hs_bits=w.B.shape[0],
                    precision=precision, k=k, hs_images=hs)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_image_calls(dev, graph):
    w = small_workload()
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs)
    got = b.run(kps, pairs, B, t, graph=graph)
    ref = single_image_outputs(w, imgs, hs, kps, pairs, B, t)
    assert_same(got, ref, f"graph={graph}")
    # the empty train set and the short one give the documented sentinels
    rows = b.match_offsets
    i_tiny = w.matches.index((2, 3))  # 37x29 scene with 40 keypoints
    assert rows[i_tiny + 1] - rows[i_tiny] == 40
    idx = to_np(got["bad_idx"])
    assert (idx[rows[i_tiny]:rows[i_tiny + 1]] >= 0).all()
    b.close()


def test_batch_with_float_hashsift_images_and_k1(dev):
    w = small_workload(seed=synth.SEED_BASE + 51, bad_bits=256, hs_bits=512)
    imgs, hs, kps, pairs, B, t = upload(w, dev, hs_f32=True)
    b = make_batch(w, imgs, hs=hs, k=1)
    got = b.run(kps, pairs, B, t)
    assert_same(got, single_image_outputs(w, imgs, hs, kps, pairs, B, t, k=1))


def test_batch_mixed_hashsift_sources(dev):
    """Float32 HashSIFT sources for some images, the u8 images (given, or
    None) for the others: the batch's mixed-dtype histogram path, equal to
    the single-image calls on each image's own source."""
    w = small_workload(seed=synth.SEED_BASE + 58)
    imgs, _, kps, pairs, B, t = upload(w, dev)
    hs = [(im.float() / 255.0).contiguous() if j % 2 == 0 else (im if j % 4 == 1 else None)
          for j, im in enumerate(imgs)]
    b = make_batch(w, imgs, hs=hs)
    got = b.run(kps, pairs, B, t)
    ref_hs = [h if h is not None else im for h, im in zip(hs, imgs)]
    assert_same(got, single_image_outputs(w, imgs, ref_hs, kps, pairs, B, t), "mixed")
    b.close()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_batch_reduced_precision_equals_single_image(dev, precision):
    w = small_workload(seed=synth.SEED_BASE + 52)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs, precision=precision)
    got = b.run(kps, pairs, B, t)
    assert_same(got, single_image_outputs(w, imgs, hs, kps, pairs, B, t, precision=precision), precision)


def test_batch_outputs_do_not_depend_on_tuning(dev):
    w = small_workload(seed=synth.SEED_BASE + 53)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs)
    ref = b.run(kps, pairs, B, t, graph=False)
    tunings = [
        dict(order_blocks_per_cu=1, integral_blocks_per_cu=1, bad_blocks_per_cu=1, hist_blocks_per_cu=1,
             knn_qpl=[1, 1], knn_rows=[256, 256], knn_blocks_per_cu=[1, 1]),
        dict(integral_blocks_per_cu=16, bad_blocks_per_cu=16, hist_blocks_per_cu=8,
             knn_qpl=[2, 4], knn_rows=[4096, 512], knn_blocks_per_cu=[8, 2]),
        dict(knn_qpl=[4, 2], knn_rows=[1 << 22, 300], knn_blocks_per_cu=[16, 16]),
        # the MFMA engine: one-unit splits, several per problem, one for all
        dict(knn_qpl=[0, 0], knn_rows=[256, 272], knn_blocks_per_cu=[1, 3]),
        dict(knn_qpl=[0, 1], knn_rows=[2048, 1024], knn_blocks_per_cu=[2, 4]),
    ]
    for tn in tunings:
        b.tuning = tn
        assert_same(b.run(kps, pairs, B, t), ref, str(tn))


def test_batch_graph_replays_match_eager(dev):
    """Replays of the captured graph, with other eager work and synchronizations
    in between, each equal the eager result; new output buffers recapture."""
    w = small_workload(seed=synth.SEED_BASE + 54)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs)
    ref = b.run(kps, pairs, B, t, graph=False)
    out = b.allocate_outputs()
    for rep in range(3):
        for v in out.values():
            v.fill_(7)  # eager work that must not leak into the replay
        b.run(kps, pairs, B, t, out=out, graph=True)
        torch.cuda.synchronize()
        assert_same(out, ref, f"replay {rep}")
    assert_same(b.run(kps, pairs, B, t, graph=True), ref, "new outputs")


def test_batch_autotune_keeps_results(dev):
    w = small_workload(seed=synth.SEED_BASE + 55)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs)
    ref = b.run(kps, pairs, B, t, graph=False)
    out = b.allocate_outputs()
    tn = b.autotune(kps, pairs, B, t, out=out, reps=1)
    assert tn["knn_qpl"][0] in (0, 1, 2, 4) and tn["knn_rows"][0] >= 256
    assert_same(out, ref, "autotune outputs")
    assert_same(b.run(kps, pairs, B, t), ref, "after autotune")


def test_batch_sample_against_oracle(dev, ref):
    """Codes of sampled keypoints of two images against the oracle directly."""
    w = small_workload(seed=synth.SEED_BASE + 56)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    got = make_batch(w, imgs).run(kps, pairs, B, t)
    offs = np.concatenate([[0], np.cumsum([len(x) for x in w.kps])])
    rng = np.random.default_rng(5)
    for j in (0, 7):
        sel = np.sort(rng.choice(len(w.kps[j]), 60, replace=False))
        kp = w.kps[j][sel]
        ii = ref.build_integral(w.images[j])
        codes, _ = ref.describe_bad(ii, kp, w.pairs)
        np.testing.assert_array_equal(to_np(got["bad_codes"])[offs[j] + sel], codes)
        _, resp, hcodes = ref.describe_hashsift(w.images[j], kp, w.B, w.t)
        gbits = np.unpackbits(to_np(got["hs_codes"])[offs[j] + sel].view(np.uint8), axis=1, bitorder="little")
        obits = np.unpackbits(hcodes.view(np.uint8), axis=1, bitorder="little")
        safe = np.abs(resp) >= 2e-4
        np.testing.assert_array_equal(gbits[safe], obits[safe])


def test_batch_validation_errors(dev):
    w = small_workload(seed=synth.SEED_BASE + 57, sizes=[(64, 48, 10)])
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    with pytest.raises(bd.BDError, match="0, 256 or 512"):
        bd.Batch(imgs, [10, 10], w.matches, bad_bits=128)
    with pytest.raises(bd.BDError, match="names image"):
        bd.Batch(imgs, [10, 10], [(0, 5)])
    b = make_batch(w, imgs)
    with pytest.raises(bd.BDError, match="rows per unit"):
        b.tuning = dict(knn_rows=[100, 1024])
    with pytest.raises(bd.BDError, match="queries per lane"):
        b.tuning = dict(knn_qpl=[3, 1])
    with pytest.raises(bd.BDError, match="multiple of 16"):
        b.tuning = dict(knn_qpl=[0, 1], knn_rows=[300, 1024])
    with pytest.raises(bd.BDError, match="up to 2048"):
        b.tuning = dict(knn_qpl=[1, 0], knn_rows=[1024, 2048 + 16])
    # a rejected tuning leaves the batch usable
    assert_same(b.run(kps, pairs, B, t), single_image_outputs(w, imgs, hs, kps, pairs, B, t))


def test_batched_workload_full_size(dev, ref):
    """The 64-scene workload (128 images, 320x240 .. 4000x3000, 500 .. 20000
    keypoints, BAD-512 + HashSIFT-256, 2-NN against each copy) in the launch
    configuration the benchmark times: autotuned and replayed as a graph,
    checked against the single-image calls on every image, and the largest
    scene (both views, every keypoint) against the oracle directly: BAD-512
    codes bit for bit, HashSIFT-256 bits wherever the FP64 response is at
    least 2e-4 from its threshold, and the BAD 2-NN of 1000 sampled queries
    bit for bit."""
    w = synth.batched()
    print(f"\n[batched full] {len(w.images)} images, {w.total_kp} keypoints", flush=True)
    imgs, hs, kps, pairs, B, t = upload(w, dev)
    b = make_batch(w, imgs)
    out = b.allocate_outputs()
    b.autotune(kps, pairs, B, t, out=out, reps=1)
    got = b.run(kps, pairs, B, t, out=out, graph=True)
    ref_out = single_image_outputs(w, imgs, hs, kps, pairs, B, t)
    assert_same(got, ref_out, "full")
    match_rows = list(b.match_offsets)
    b.close()

    offs = np.concatenate([[0], np.cumsum([len(x) for x in w.kps])])
    m = max(range(len(w.matches)), key=lambda i: w.images[w.matches[i][0]].size)
    qi, ti = w.matches[m]
    H, W = w.images[qi].shape
    print(f"[batched full] oracle check of scene {m}: {W}x{H}, {len(w.kps[qi])} keypoints per view", flush=True)
    bad_ref = {}
    for j in (qi, ti):
        ii = ref.build_integral(w.images[j])
        codes, _ = ref.describe_bad(ii, w.kps[j], w.pairs)
        np.testing.assert_array_equal(to_np(got["bad_codes"])[offs[j]:offs[j + 1]], codes, err_msg=f"BAD image {j}")
        bad_ref[j] = codes
        _, resp, hcodes = ref.describe_hashsift(w.images[j], w.kps[j], w.B, w.t)
        gbits = np.unpackbits(to_np(got["hs_codes"])[offs[j]:offs[j + 1]].view(np.uint8), axis=1, bitorder="little")
        obits = np.unpackbits(hcodes.view(np.uint8), axis=1, bitorder="little")
        safe = np.abs(resp) >= 2e-4
        assert safe.mean() > 0.99
        np.testing.assert_array_equal(gbits[safe], obits[safe], err_msg=f"HashSIFT image {j}")
    # 2-NN of 1000 sampled queries against the whole train view (each query is
    # independent, so the sample is checked exactly)
    sel = np.sort(np.random.default_rng(6).choice(len(w.kps[qi]), min(1000, len(w.kps[qi])), replace=False))
    ei, ed = ref.match_knn(bad_ref[qi][sel], bad_ref[ti], 2)
    lo = int(match_rows[m])
    assert int(match_rows[m + 1]) - lo == len(w.kps[qi])
    np.testing.assert_array_equal(to_np(got["bad_idx"])[lo + sel], ei)
    np.testing.assert_array_equal(to_np(got["bad_dist"])[lo + sel], ed)

