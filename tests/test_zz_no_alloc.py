"""bd_match_hamming_knn_noalloc through the C ABI: the same indices and
distances, bit for bit, as bd_match_hamming_knn on the same inputs, for two
calls in a row (the second smaller, so it runs over the first call's stale
scratch contents), plus an oracle check of the first call and the rejection
of a problem whose partial keys exceed the fixed scratch array."""

import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu


def _abi_call(fn, ctx, q, t, k, stream):
    n_q, n_words = q.shape
    idx = torch.full((n_q, k), -7, dtype=torch.int32, device=q.device)
    dist = torch.full((n_q, k), 7, dtype=torch.uint32, device=q.device)
    rc = fn(ctx, q.data_ptr(), n_q, t.data_ptr(), t.shape[0], n_words, k, idx.data_ptr(), dist.data_ptr(), stream)
    assert rc == bd.BD_OK, bd.last_error()
    return to_np(idx), to_np(dist)


@pytest.mark.parametrize("first,second", [((5000, 5000, 4, 2), (1000, 3000, 8, 1)),
                                          ((3000, 20000, 8, 2), (64, 100, 4, 2)),
                                          ((2000, 1500, 3, 2), (17, 5, 3, 1))])
def test_noalloc_equals_allocating_entry_point(ref, dev, first, second):
    L = bd.lib()
    stream = torch.cuda.current_stream(dev).cuda_stream
    ctx = bd.context(dev.index, stream)
    rng = np.random.default_rng(sum(first) * 7 + sum(second))
    for call, (n_q, n_t, n_words, k) in enumerate((first, second)):
        print(f"no-alloc k-NN call {call}: n_q={n_q} n_t={n_t} n_words={n_words} k={k}", flush=True)
        t_np = synth.random_codes(rng, n_t, n_words)
        q_np = synth.random_codes(rng, n_q, n_words)
        q_np[: n_q // 4] = t_np[rng.integers(0, n_t, n_q // 4)]  # exact duplicates and ties
        t_np[n_t // 2:n_t // 2 + 3] = t_np[1]
        q = torch.from_numpy(q_np).to(dev)
        t = torch.from_numpy(t_np).to(dev)
        gi, gd = _abi_call(L.bd_match_hamming_knn_noalloc, ctx, q, t, k, stream)
        ei, ed = _abi_call(L.bd_match_hamming_knn, ctx, q, t, k, stream)
        np.testing.assert_array_equal(gi, ei)
        np.testing.assert_array_equal(gd, ed)
        if call == 0:
            ri, rd = ref.match_knn(q_np[:500], t_np, k)
            np.testing.assert_array_equal(gi[:500], ri)
            np.testing.assert_array_equal(gd[:500], rd)


def test_noalloc_binding_and_empty_queries(ref, dev):
    stream = torch.cuda.current_stream(dev).cuda_stream
    bd.context(dev.index, stream)
    rng = np.random.default_rng(11)
    q_np = synth.random_codes(rng, 300, 4)
    t_np = synth.random_codes(rng, 1, 4)
    q = torch.from_numpy(q_np).to(dev)
    t = torch.from_numpy(t_np).to(dev)
    idx = torch.empty((300, 2), dtype=torch.int32, device=dev)
    dist = torch.empty((300, 2), dtype=torch.uint32, device=dev)
    bd.match_hamming_knn_noalloc(q, t, idx, dist)
    ri, rd = ref.match_knn(q_np, t_np, 2)  # n_t < k: the second slot is empty
    np.testing.assert_array_equal(to_np(idx), ri)
    np.testing.assert_array_equal(to_np(dist), rd)
    e_idx = torch.empty((0, 1), dtype=torch.int32, device=dev)
    e_dist = torch.empty((0, 1), dtype=torch.uint32, device=dev)
    bd.match_hamming_knn_noalloc(q[:0], t, e_idx, e_dist)


def test_noalloc_rejects_problems_beyond_the_scratch(dev):
    """100 000 x 200 000 2-NN needs 98 splits x 100 000 x 2 keys (78 MB): BD_EINVAL
    before anything is enqueued.  The buffers are full-size all the same."""
    L = bd.lib()
    stream = torch.cuda.current_stream(dev).cuda_stream
    ctx = bd.context(dev.index, stream)
    n_q, n_t, k = 100_000, 200_000, 2
    q = torch.zeros((n_q, 4), dtype=torch.uint64, device=dev)
    t = torch.zeros((n_t, 4), dtype=torch.uint64, device=dev)
    idx = torch.zeros((n_q, k), dtype=torch.int32, device=dev)
    dist = torch.zeros((n_q, k), dtype=torch.uint32, device=dev)
    rc = L.bd_match_hamming_knn_noalloc(ctx, q.data_ptr(), n_q, t.data_ptr(), n_t, 4, k, idx.data_ptr(),
                                        dist.data_ptr(), stream)
    assert rc == bd.BD_EINVAL
    assert "scratch" in bd.last_error()
    torch.cuda.synchronize()
    assert int(idx.abs().sum()) == 0  # nothing ran
