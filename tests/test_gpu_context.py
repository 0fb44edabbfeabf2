"""bd_context_poll: the describe calls of a context count the invalid
keypoints they meet (a non-finite field or scale <= 0, Sec. III-A/III-B give
such a keypoint no patch), the poll returns the count and resets it.  Each
case runs on its own stream, hence on a fresh context of the binding."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu

BAD_ROWS = [3, 50, 51, 199, 298]


def workload():
    w = synth.hashsift512_pair(synth.SEED_BASE + 77, width=320, height=240, n_kp=300, n_bits=256, with_bad_bits=256)
    kp = w.kp1.copy()
    kp["x"][3] = np.nan
    kp["y"][50] = np.inf
    kp["scale"][51] = 0.0
    kp["scale"][199] = -1.5
    kp["angle"][298] = -np.inf
    return w, kp


def test_poll_counts_invalid_keypoints_per_describe_call(dev):
    w, kp = workload()
    s = torch.cuda.Stream(dev)
    with torch.cuda.stream(s):
        stream = s.cuda_stream
        assert bd.context_poll(dev.index, stream) == 0
        img = torch.from_numpy(w.extra["image1_u8"]).to(dev)
        kps = bd.keypoints_tensor(kp, dev)
        pairs = bd.pairs_tensor(w.pairs, dev)
        B = torch.from_numpy(w.B).to(dev)
        t = torch.from_numpy(w.t).to(dev)
        ii = bd.build_integral(img)
        assert bd.context_poll(dev.index, stream) == 0  # the integral image has no keypoints

        bad = bd.describe_bad(ii, kps, pairs)
        assert bd.context_poll(dev.index, stream) == len(BAD_ROWS)
        assert bd.context_poll(dev.index, stream) == 0  # reset by the poll
        assert not to_np(bad)[BAD_ROWS].any()

        table = bd.BadTable(pairs)
        bd.describe_bad(ii, kps, table=table)
        order = bd.keypoint_order(kps, img.shape[1], img.shape[0])
        bd.describe_bad(ii, kps, pairs, order=order)
        assert bd.context_poll(dev.index, stream) == 2 * len(BAD_ROWS)
        table.close()

        codes, hist, _ = bd.describe_hashsift(torch.from_numpy(w.image1).to(dev), kps, B, t, with_hist=True,
                                              with_resp=True)
        assert bd.context_poll(dev.index, stream) == len(BAD_ROWS)  # once per keypoint, not per stage
        assert not to_np(codes)[BAD_ROWS].any() and not to_np(hist)[BAD_ROWS].any()

        bd.hashsift_features(img, kps)
        bd.hashsift_project(hist, B, t, kps=kps)  # masks codes, does not count
        assert bd.context_poll(dev.index, stream) == len(BAD_ROWS)

        valid = bd.keypoints_tensor(w.kp1, dev)
        bd.describe_bad(ii, valid, pairs)
        bd.describe_hashsift(img, valid, B, t)
        assert bd.context_poll(dev.index, stream) == 0


def test_poll_counts_the_batch_stages(dev):
    w = synth.batched(synth.SEED_BASE + 51, sizes=[(320, 240, 200), (200, 150, 90)])
    flat = w.flat_keypoints().copy()
    flat["x"][[0, 7, 250]] = np.nan
    imgs = [torch.from_numpy(np.ascontiguousarray(im)).to(dev) for im in w.images]
    kps = bd.keypoints_tensor(flat, dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    B = torch.from_numpy(w.B).to(dev)
    t = torch.from_numpy(w.t).to(dev)
    b = bd.Batch(imgs, [len(x) for x in w.kps], w.matches, bad_bits=w.pairs.shape[0], hs_bits=B.shape[0])
    bd.context_poll(dev.index)  # the batch's context may carry counts of earlier calls
    out = b.run(kps, pairs, B, t, graph=False)
    assert bd.context_poll(dev.index) == 2 * 3  # BAD and HashSIFT stages
    assert not to_np(out["bad_codes"])[[0, 7, 250]].any()
    b.run(kps, pairs, B, t, graph=True)
    assert bd.context_poll(dev.index) == 2 * 3
    b.close()


def test_workspace_allocation_failure_reports_enomem(dev, monkeypatch):
    """With BD_TEST_FAIL_ALLOC=1 the workspace allocation of a fresh context
    fails: the call returns BD_ENOMEM with a message and enqueues nothing;
    without it the same call on the same context succeeds."""
    rng = np.random.default_rng(5)
    q = torch.from_numpy(synth.random_codes(rng, 5000, 4)).to(dev)
    t = torch.from_numpy(synth.random_codes(rng, 5000, 4)).to(dev)  # several splits: needs workspace
    ref_idx, ref_dist = bd.match_hamming_knn(q, t, k=2)
    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        monkeypatch.setenv("BD_TEST_FAIL_ALLOC", "1")
        idx = torch.full((5000, 2), -5, dtype=torch.int32, device=dev)
        dist = torch.zeros((5000, 2), dtype=torch.uint32, device=dev)
        with pytest.raises(bd.BDError) as e:
            bd.match_hamming_knn(q, t, k=2, idx=idx, dist=dist)
        assert e.value.code == bd.BD_ENOMEM and "injected" in str(e.value)
        assert (to_np(idx) == -5).all()
        monkeypatch.delenv("BD_TEST_FAIL_ALLOC")
        bd.match_hamming_knn(q, t, k=2, idx=idx, dist=dist)
        np.testing.assert_array_equal(to_np(idx), to_np(ref_idx))
        np.testing.assert_array_equal(to_np(dist), to_np(ref_dist))
