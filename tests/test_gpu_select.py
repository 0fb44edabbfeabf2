"""Alg. 2 threshold search on the GPU against the oracle: best bin, loss and
threshold of every candidate bit-exact (integer bins, half-integer losses)."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth

from conftest import to_np

pytestmark = pytest.mark.gpu


def triplet_patches(seed, n):
    b = synth.triplets(seed, n=n)
    p = np.empty((3 * n, 32, 32), dtype=np.float32)
    p[0::3], p[1::3], p[2::3] = b.anchor, b.positive, b.negative
    return np.clip(np.rint(p * 255.0), 0, 255).astype(np.uint8)


def run_both(ref, dev, patches, s_ap, s_an, tau, cands):
    eb, el = ref.find_threshold(patches, s_ap, s_an, tau, cands)
    gb, gt, gl = bd.find_threshold(torch.from_numpy(patches).to(dev), torch.from_numpy(s_ap).to(dev),
                                   torch.from_numpy(s_an).to(dev), tau, bd.pairs_tensor(cands, dev))
    np.testing.assert_array_equal(to_np(gb), eb)
    np.testing.assert_array_equal(to_np(gl), el)
    np.testing.assert_array_equal(to_np(gt), ((eb.astype(np.float64) + 1 - 2550) / 10.0).astype(np.float32))
    return eb, el


@pytest.mark.parametrize("n,J,tau", [(1, 3, 0.5), (5, 9, 1.0), (37, 100, 0.5), (400, 257, 2.0), (2001, 64, 1.5)])
def test_find_threshold_equals_oracle(ref, dev, n, J, tau):
    rng = np.random.default_rng(n + J)
    patches = triplet_patches(synth.SEED_BASE + 60 + n, n)
    if n >= 5:
        patches[3] = patches[4]   # ties inside a triplet
        patches[9:12] = 77        # a constant triplet
    K = 31
    s_ap = rng.integers(-K, K + 1, n).astype(np.int32)
    s_an = rng.integers(-K, K + 1, n).astype(np.int32)
    cands = synth.box_pairs(rng, J, max_offset=15, radius_range=(0, 15))
    run_both(ref, dev, patches, s_ap, s_an, tau, cands)


def test_first_selection_step(ref, dev):
    """The first round of the greedy selection (no bits yet: s = 0) on 4096
    triplets with 1000 candidates, the paper's J (Sec. III-A)."""
    n, J = 4096, 1000
    rng = np.random.default_rng(61)
    patches = triplet_patches(synth.SEED_BASE + 61, n)
    zeros = np.zeros(n, dtype=np.int32)
    cands = synth.box_pairs(rng, J, max_offset=14, radius_range=(0, 7))
    eb, el = run_both(ref, dev, patches, zeros, zeros, 1.0, cands)
    # loss at the lowest threshold is n * [1 - 1 + 1]_+ = n; the best candidates do better
    assert el.max() <= n and el.min() < 0.9 * n


def test_no_triplets(dev):
    cands = bd.pairs_tensor(synth.box_pairs(np.random.default_rng(1), 5), dev)
    empty = torch.zeros((0,), dtype=torch.int32, device=dev)
    b, t, l = bd.find_threshold(torch.zeros((0, 32, 32), dtype=torch.uint8, device=dev), empty, empty, 0.5, cands)
    assert (to_np(b) == 0).all() and (to_np(l) == 0).all()
