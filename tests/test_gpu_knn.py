"""Hamming k-NN on the GPU against the oracle, bit for bit (indices and distances)."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu


def both(ref, dev, q, t, k):
    ei, ed = ref.match_knn(q, t, k)
    gi, gd = bd.match_hamming_knn(torch.from_numpy(q).to(dev), torch.from_numpy(t).to(dev), k)
    return to_np(gi), to_np(gd), ei, ed


@pytest.mark.parametrize("n_words", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("k", [1, 2])
def test_random_codes_with_ties(ref, dev, n_words, k):
    rng = np.random.default_rng(n_words * 10 + k)
    t = synth.random_codes(rng, 777, n_words)
    t[100:110] = t[5]  # runs of equal codes: ties resolved by lower index
    q = synth.random_codes(rng, 333, n_words)
    q[:20] = t[5]
    q[20:40] ^= q[20:40] & np.uint64(0xF)  # near-duplicates
    gi, gd, ei, ed = both(ref, dev, q, t, k)
    np.testing.assert_array_equal(gi, ei)
    np.testing.assert_array_equal(gd, ed)


@pytest.mark.parametrize("n_q,n_t", [(1, 1), (1, 2), (2, 1), (63, 64), (65, 63), (1000, 1000), (64, 5000),
                                     (5000, 17), (3, 200000)])
def test_shapes_and_split_paths(ref, dev, n_q, n_t):
    """Small train sets run in one split (direct write); large ones split and merge."""
    rng = np.random.default_rng(n_q * 31 + n_t)
    q = synth.random_codes(rng, n_q, 4)
    t = synth.random_codes(rng, n_t, 4)
    t[n_t // 2] = q[0]
    gi, gd, ei, ed = both(ref, dev, q, t, 2)
    np.testing.assert_array_equal(gi, ei)
    np.testing.assert_array_equal(gd, ed)


def test_fewer_train_codes_than_k(ref, dev):
    rng = np.random.default_rng(3)
    q = synth.random_codes(rng, 70, 8)
    gi, gd, ei, ed = both(ref, dev, q, q[:1], 2)
    np.testing.assert_array_equal(gi, ei)
    np.testing.assert_array_equal(gd, ed)
    gi, gd = bd.match_hamming_knn(torch.from_numpy(q).to(dev), torch.zeros((0, 8), dtype=torch.uint64, device=dev), 2)
    assert (to_np(gi) == -1).all() and (to_np(gd) == 0xFFFFFFFF).all()


def test_empty_query_set(dev):
    t = torch.zeros((5, 4), dtype=torch.uint64, device=dev)
    gi, gd = bd.match_hamming_knn(torch.zeros((0, 4), dtype=torch.uint64, device=dev), t, 1)
    assert gi.shape == (0, 1)


def test_extreme_distances(ref, dev):
    rng = np.random.default_rng(4)
    q = synth.random_codes(rng, 50, 8)
    gi, gd, ei, ed = both(ref, dev, q, ~q, 1)
    assert (gd == 512).all() or (gd <= 512).all()
    np.testing.assert_array_equal(gd, ed)
    np.testing.assert_array_equal(gi, ei)


@pytest.mark.parametrize("n_words,k,n", [(4, 1, 1000), (8, 2, 5000)])
def test_config_sizes(ref, dev, n_words, k, n):
    """1000 x 1000 BAD-256 1-NN and 5000 x 5000 HashSIFT-512 2-NN shapes."""
    rng = np.random.default_rng(n)
    q = synth.random_codes(rng, n, n_words)
    t = q ^ (synth.random_codes(rng, n, n_words) & synth.random_codes(rng, n, n_words) & synth.random_codes(rng, n, n_words))
    gi, gd, ei, ed = both(ref, dev, q, t, k)
    np.testing.assert_array_equal(gi, ei)
    np.testing.assert_array_equal(gd, ed)


def test_deterministic(dev):
    rng = np.random.default_rng(5)
    q = torch.from_numpy(synth.random_codes(rng, 3000, 8)).to(dev)
    t = torch.from_numpy(synth.random_codes(rng, 4000, 8)).to(dev)
    a = [to_np(x) for x in bd.match_hamming_knn(q, t, 2)]
    b = [to_np(x) for x in bd.match_hamming_knn(q, t, 2)]
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_train_set_beyond_packed_row_range(ref, dev):
    """More than 2^22 train codes: the row index no longer fits the 22 bits of
    a packed key, so the set is split and merged with global indices.  Exact
    duplicates of the queries are planted on both sides of row 2^22 (ties
    resolved to the lower index) and near-duplicates beyond it."""
    rng = np.random.default_rng(78)
    n_t = (1 << 22) + 3000
    q = rng.integers(0, 2**63, (100, 1), dtype=np.uint64)
    t = rng.integers(0, 2**63, (n_t, 1), dtype=np.uint64)
    t[(1 << 22) + 5] = q[0]
    t[(1 << 22) - 7] = q[0]
    t[(1 << 22) + 100] = q[1]
    t[n_t - 1] = q[2] ^ np.uint64(1)
    t[(1 << 22) + 200] = q[3]
    t[17] = q[3] ^ np.uint64(3)
    for k in (1, 2):
        idx, dist = bd.match_hamming_knn(torch.from_numpy(q).to(dev), torch.from_numpy(t).to(dev), k=k)
        ei, ed = ref.match_knn(q, t, k)
        np.testing.assert_array_equal(to_np(idx), ei)
        np.testing.assert_array_equal(to_np(dist), ed)
    assert ei[0, 0] == (1 << 22) - 7 and ei[1, 0] == (1 << 22) + 100 and ei[2, 0] == n_t - 1


@pytest.mark.parametrize("n_words", [4, 8])
@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("n_q,n_t", [(15, 63), (16, 64), (17, 65), (31, 95), (33, 97), (255, 129), (256, 300),
                                     (257, 1031)])
def test_mfma_tile_and_chunk_boundaries(ref, dev, n_words, k, n_q, n_t):
    """Codes of 4 and 8 words run on the int8 MFMA engine (32-query x 32-row
    tiles, 64-row LDS chunks, 256 queries per block): query and train counts
    around those sizes, with equal codes planted across tiles and chunks so
    ties must resolve to the lower index, and a partial last chunk."""
    rng = np.random.default_rng(n_q * 7 + n_t * 3 + n_words + k)
    t = synth.random_codes(rng, n_t, n_words)
    q = synth.random_codes(rng, n_q, n_words)
    for j, r in enumerate(sorted({0, 15, 16, 63, 64, n_t - 1} & set(range(n_t)))):
        t[r] = q[j % n_q]                      # exact matches in different tiles and chunks
    t[n_t - 1] = t[min(15, n_t - 1)]          # a tie between the first and the last chunk
    q[n_q - 1] = t[n_t // 2] ^ np.uint64(1)    # a near match in the middle
    gi, gd, ei, ed = both(ref, dev, q, t, k)
    np.testing.assert_array_equal(gd, ed)
    np.testing.assert_array_equal(gi, ei)


def test_mfma_train_set_beyond_packed_row_range(ref, dev):
    """4-word codes (MFMA engine) with more than 2^22 train codes: splits and
    the merge restore global indices; duplicates on both sides of 2^22."""
    rng = np.random.default_rng(79)
    n_t = (1 << 22) + 1000
    q = synth.random_codes(rng, 8, 4)
    t = synth.random_codes(rng, n_t, 4)
    t[(1 << 22) + 5] = q[0]
    t[(1 << 22) - 7] = q[0]
    t[(1 << 22) + 100] = q[1]
    t[n_t - 1] = q[2] ^ np.uint64(1)
    for k in (1, 2):
        idx, dist = bd.match_hamming_knn(torch.from_numpy(q).to(dev), torch.from_numpy(t).to(dev), k=k)
        ei, ed = ref.match_knn(q, t, k)
        np.testing.assert_array_equal(to_np(dist), ed)
        np.testing.assert_array_equal(to_np(idx), ei)
    assert ei[0, 0] == (1 << 22) - 7 and ei[1, 0] == (1 << 22) + 100 and ei[2, 0] == n_t - 1


def test_mfma_splits_of_full_tag_range(ref, dev):
    """8-word codes, few queries and 2^21 + 100 train codes: the plan cuts the
    train set into splits of bd.MFMA_MAX_ROWS rows (2048: 64 tiles of 32 rows,
    the most the key's 6-bit tile tag covers), so tags 0 and 63 both occur;
    duplicates planted across a split boundary and across the first and the
    last tile of one split must resolve to the lower index."""
    rng = np.random.default_rng(83)
    S, T = bd.MFMA_MAX_ROWS, 32
    n_t = (1 << 21) + 100
    q = synth.random_codes(rng, 8, 8)
    t = synth.random_codes(rng, n_t, 8)
    t[S * 5 + S - 1] = q[0]               # last row of a split (tag 63)
    t[S * 6] = q[0]                       # first row of the next split (tag 0)
    t[S * 9 + T - 1] = q[1] ^ np.uint64(1)                 # last row of tile 0 of split 9
    t[S * 9 + (S // T - 1) * T] = q[1] ^ np.uint64(2)      # first row of tile 63 of split 9: a tie
    t[S * 11 + 3] = q[3] ^ np.uint64(4)                    # tile 0 ...
    t[S * 11 + S - 2] = q[3] ^ np.uint64(8)                # ... against tile 63, second neighbour
    t[n_t - 1] = q[2]
    t[n_t - 100] = q[2]
    for k in (1, 2):
        idx, dist = bd.match_hamming_knn(torch.from_numpy(q).to(dev), torch.from_numpy(t).to(dev), k=k)
        ei, ed = ref.match_knn(q, t, k)
        np.testing.assert_array_equal(to_np(dist), ed)
        np.testing.assert_array_equal(to_np(idx), ei)
    assert ei[0, 0] == S * 5 + S - 1 and ei[1, 0] == S * 9 + T - 1 and ei[2, 0] == n_t - 100
    assert ei[1, 1] == S * 9 + (S // T - 1) * T and ei[3, 0] == S * 11 + 3 and ei[3, 1] == S * 11 + S - 2
