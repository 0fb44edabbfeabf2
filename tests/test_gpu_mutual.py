"""Mutual nearest neighbours with the distance-ratio filter on the GPU
against the oracle: match indices, distances and counts bit-exact, ratios
equal to the oracle's double ratio rounded to float32."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth

from conftest import to_np

pytestmark = pytest.mark.gpu


def noisy_pair(rng, n_q, n_t, nw, flip=0.08):
    q = rng.integers(0, 2**63, (n_q, nw), dtype=np.uint64)
    src = q[rng.integers(0, n_q, n_t)] if n_q else rng.integers(0, 2**63, (n_t, nw), dtype=np.uint64)
    bits = np.unpackbits(src.view(np.uint8), axis=1)
    bits ^= (rng.random(bits.shape) < flip).astype(np.uint8)
    t = np.packbits(bits, axis=1).view(np.uint64).reshape(n_t, nw)
    if n_t > 4:
        t[1] = t[0]  # exact duplicates: ties in both directions and d1 == d2
    return q, t


CASES = [(1, 1, 1), (2, 3, 4), (63, 65, 4), (700, 513, 8), (1000, 1000, 4), (300, 5000, 8), (4097, 129, 2), (5, 0, 4)]


@pytest.mark.parametrize("n_q,n_t,nw", CASES)
@pytest.mark.parametrize("max_ratio", [0.0, 0.8])
def test_mutual_equals_oracle(dev, ref, n_q, n_t, nw, max_ratio):
    rng = np.random.default_rng(n_q * 7 + n_t + nw)
    q, t = noisy_pair(rng, n_q, n_t, nw)
    r32 = float(np.float32(max_ratio))
    m_ref, d_ref, ratio_ref, c_ref = ref.match_mutual(q, t, r32)
    match, dist, ratio, count = bd.match_mutual(torch.from_numpy(q).to(dev), torch.from_numpy(t).to(dev),
                                                r32, with_ratio=True, with_count=True)
    np.testing.assert_array_equal(to_np(match), m_ref)
    np.testing.assert_array_equal(to_np(dist), d_ref)
    np.testing.assert_array_equal(to_np(ratio), ratio_ref.astype(np.float32))
    assert int(to_np(count)[0]) == c_ref


def test_mutual_on_described_views(dev, ref):
    """BAD-256 codes of the two views of the plain workload: MNN + ratio 0.8
    keeps mostly true correspondences (keypoint i of view 1 is keypoint i of
    view 2), and equals the oracle on the GPU's own codes."""
    w = synth.bad256_pair()
    img1 = torch.from_numpy(w.image1).to(dev)
    img2 = torch.from_numpy(w.image2).to(dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    c1 = bd.describe_bad(bd.build_integral(img1), bd.keypoints_tensor(w.kp1, dev), pairs)
    c2 = bd.describe_bad(bd.build_integral(img2), bd.keypoints_tensor(w.kp2, dev), pairs)
    r32 = float(np.float32(0.8))
    match, dist, count = bd.match_mutual(c1, c2, r32, with_count=True)
    m_ref, d_ref, _, c_ref = ref.match_mutual(to_np(c1), to_np(c2), r32)
    np.testing.assert_array_equal(to_np(match), m_ref)
    np.testing.assert_array_equal(to_np(dist), d_ref)
    m = to_np(match)
    kept = m >= 0
    assert int(to_np(count)[0]) == c_ref == kept.sum() > 500
    assert (m[kept] == np.arange(len(m))[kept]).mean() > 0.99


def test_mutual_count_only_for_empty_queries(dev):
    q = torch.zeros((0, 4), dtype=torch.uint64, device=dev)
    t = torch.zeros((3, 4), dtype=torch.uint64, device=dev)
    match, dist, count = bd.match_mutual(q, t, 0.8, with_count=True)
    assert match.numel() == 0 and int(to_np(count)[0]) == 0
