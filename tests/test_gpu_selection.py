"""Greedy BAD feature selection (Alg. 1) on the GPU against the oracle: the
chosen candidate, bin and loss of every round, the table and the pool codes
bit-exact."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth

from conftest import to_np

pytestmark = pytest.mark.gpu


def pool_of(seed, P):
    b = synth.triplets(seed, n=P)
    pool = np.empty((2 * P, 32, 32), dtype=np.uint8)
    pool[0::2] = np.clip(np.rint(b.anchor * 255), 0, 255)
    pool[1::2] = np.clip(np.rint(b.positive * 255), 0, 255)
    return pool


@pytest.mark.parametrize("P,N,J,K,tau", [(12, 2, 3, 3, 0.5), (300, 200, 64, 70, 1.0), (150, 150, 1000, 3, 2.0)])
def test_selection_equals_oracle(ref, dev, P, N, J, K, tau):
    rng = np.random.default_rng(P + N + J + K)
    pool = pool_of(synth.SEED_BASE + 70 + P, P)
    samples = np.stack([rng.permutation(P)[:N] for _ in range(K)]).astype(np.int32)
    cands = np.stack([synth.box_pairs(rng, J, max_offset=15, radius_range=(0, 8)) for _ in range(K)])
    et, ec, eb, el, ecodes = ref.select_features(pool, samples, cands, tau)
    gt, gc, gb, gl, gcodes = bd.select_features(torch.from_numpy(pool).to(dev), torch.from_numpy(samples).to(dev),
                                                torch.from_numpy(cands.view(np.uint8).reshape(K, J, 12)).to(dev), tau)
    np.testing.assert_array_equal(to_np(gc), ec)
    np.testing.assert_array_equal(to_np(gb), eb)
    np.testing.assert_array_equal(to_np(gl), el)
    np.testing.assert_array_equal(to_np(gt), et.view(np.uint8).reshape(K, 12))
    np.testing.assert_array_equal(to_np(gcodes), ecodes)
    assert (np.diff(ec) != 0).any() or K < 3  # not a degenerate run


def test_selected_table_describes_like_bad(ref, dev):
    """The learned table used as a BAD table on the patches themselves (keypoint at
    the patch centre, scale 1, angle 0) reproduces the pool codes of the run."""
    P, N, J, K = 64, 64, 100, 256
    rng = np.random.default_rng(5)
    pool = pool_of(synth.SEED_BASE + 75, P)
    samples = np.stack([rng.permutation(P)[:N] for _ in range(K)]).astype(np.int32)
    cands = np.stack([synth.box_pairs(rng, J, radius_range=(0, 5)) for _ in range(K)])
    table, _, _, _, codes = bd.select_features(torch.from_numpy(pool).to(dev), torch.from_numpy(samples).to(dev),
                                               torch.from_numpy(cands.view(np.uint8).reshape(K, J, 12)).to(dev), 1.0)
    kp = torch.tensor([[15.5, 15.5, 1.0, 0.0]], dtype=torch.float32, device=dev)
    tab = table.contiguous()
    for x in range(0, 2 * P, 7):
        img = torch.from_numpy(pool[x]).to(dev)
        c = bd.describe_bad(bd.build_integral(img), kp, tab)
        # BAD centres at floor(15.5 + u + 0.5) = 16 + u, the patch geometry of the selection
        np.testing.assert_array_equal(to_np(c)[0], to_np(codes)[x])
