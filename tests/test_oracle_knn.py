"""Pins for the oracle's brute-force Hamming k-NN (Sec. III-A: similarity
S(x, y) = h(x)^T h(y) of +-1 codes, i.e. K - 2 d_H(x, y)).

Checked against an exhaustive numpy ranking (np.unpackbits on the XOR and a
lexicographic sort), the +-1 matrix product of the paper's similarity,
metric properties through single-element train sets, and forced ties."""
import numpy as np
import pytest

from paper_2108_08380_amd import synth


def hamming_matrix(q, t):
    x = q[:, None, :] ^ t[None, :, :]
    return np.unpackbits(x.view(np.uint8), axis=2).sum(axis=2).astype(np.int64)


def numpy_knn(q, t, k):
    d = hamming_matrix(q, t)
    idx = np.full((len(q), k), -1, dtype=np.int32)
    dist = np.full((len(q), k), 0xFFFFFFFF, dtype=np.uint32)
    for i in range(len(q)):
        order = np.lexsort((np.arange(len(t)), d[i]))[:k]
        idx[i, :len(order)] = order
        dist[i, :len(order)] = d[i, order]
    return idx, dist


@pytest.mark.parametrize("n_words", [1, 4, 8])
@pytest.mark.parametrize("k", [1, 2, 5])
def test_exhaustive_with_forced_ties(ref, n_words, k):
    rng = np.random.default_rng(30 + n_words * 7 + k)
    t = synth.random_codes(rng, 64, n_words)
    t[10] = t[3]
    t[40] = t[3]  # duplicated train codes: equal distances, order by index
    t[20] = t[21]
    q = synth.random_codes(rng, 50, n_words)
    q[0] = t[3]
    q[1] = t[21]
    q[2] = t[3] ^ np.uint64(1)  # one bit away from a triplicated code
    idx, dist = ref.match_knn(q, t, k)
    e_idx, e_dist = numpy_knn(q, t, k)
    np.testing.assert_array_equal(idx, e_idx)
    np.testing.assert_array_equal(dist, e_dist)
    assert idx[0, 0] == 3 and dist[0, 0] == 0
    if k >= 2:
        assert list(idx[0, :2]) == [3, 10] and list(idx[1, :2]) == [20, 21]


def test_identity_and_complement(ref):
    rng = np.random.default_rng(31)
    t = synth.random_codes(rng, 30, 4)
    idx, dist = ref.match_knn(t, t, 1)
    np.testing.assert_array_equal(idx[:, 0], np.arange(30))
    assert not dist.any()
    comp = ~t
    for i in range(30):
        _, d = ref.match_knn(t[i:i + 1], comp[i:i + 1], 1)
        assert d[0, 0] == 256


def test_symmetry_and_triangle_inequality(ref):
    rng = np.random.default_rng(32)
    c = synth.random_codes(rng, 12, 8)

    def d(a, b):
        return int(ref.match_knn(c[a:a + 1], c[b:b + 1], 1)[1][0, 0])

    for a in range(12):
        for b in range(12):
            assert d(a, b) == d(b, a)
            for m in range(0, 12, 3):
                assert d(a, b) <= d(a, m) + d(m, b)


def test_similarity_identity_against_pm1_matmul(ref):
    """S = h(x)^T h(y) with h in {-1, +1}^K equals K - 2 d_H."""
    rng = np.random.default_rng(33)
    q = synth.random_codes(rng, 20, 4)
    t = synth.random_codes(rng, 35, 4)
    hq = 2 * np.unpackbits(q.view(np.uint8), axis=1, bitorder="little").astype(np.int64) - 1
    ht = 2 * np.unpackbits(t.view(np.uint8), axis=1, bitorder="little").astype(np.int64) - 1
    S = hq @ ht.T
    idx, dist = ref.match_knn(q, t, len(t))  # every train code, ranked
    for i in range(len(q)):
        np.testing.assert_array_equal(256 - 2 * dist[i].astype(np.int64), S[i, idx[i]])
        assert sorted(idx[i]) == list(range(len(t)))


def test_fewer_train_codes_than_k(ref):
    rng = np.random.default_rng(34)
    q = synth.random_codes(rng, 5, 4)
    idx, dist = ref.match_knn(q, q[:1], 3)
    assert (idx[:, 0] == 0).all() and (idx[:, 1:] == -1).all() and (dist[:, 1:] == 0xFFFFFFFF).all()
    idx, dist = ref.match_knn(q, q[:0], 2)
    assert (idx == -1).all() and (dist == 0xFFFFFFFF).all()


def test_popcount_against_bit_loop(ref):
    rng = np.random.default_rng(35)
    a = synth.random_codes(rng, 40, 1)
    z = np.zeros((1, 1), dtype=np.uint64)
    _, dist = ref.match_knn(a, z, 1)
    for i in range(40):
        v, c = int(a[i, 0]), 0
        while v:
            c += v & 1
            v >>= 1
        assert dist[i, 0] == c


# ---------------------------------------------------------------- mutual nearest neighbours + ratio filter


def distance_matrix(q, t):
    """All pairwise Hamming distances by unpacking bits (independent of the oracle's popcount loop)."""
    qb = np.unpackbits(q.view(np.uint8), axis=1).astype(np.int32)
    tb = np.unpackbits(t.view(np.uint8), axis=1).astype(np.int32)
    return (qb[:, None, :] != tb[None, :, :]).sum(axis=2)


def mutual_by_matrix(q, t, max_ratio):
    D = distance_matrix(q, t)
    n_q, n_t = D.shape
    match = np.full(n_q, -1, np.int32)
    for i in range(n_q):
        if n_t == 0:
            continue
        j = int(np.argmin(D[i]))  # first minimum: lowest index among ties
        if int(np.argmin(D[:, j])) != i:
            continue
        others = np.delete(D[i], j)
        if max_ratio > 0 and len(others) and not (float(D[i, j]) < max_ratio * float(others.min())):
            continue
        match[i] = j
    return match


def test_mutual_matches_by_brute_force_distance_matrix(ref):
    rng = np.random.default_rng(70)
    for n_q, n_t, nw in ((30, 40, 1), (57, 23, 2), (64, 64, 4)):
        base = rng.integers(0, 2**63, (max(n_q, n_t), nw), dtype=np.uint64)
        q = base[:n_q].copy()
        t = base[rng.permutation(len(base))[:n_t]].copy()
        t ^= (rng.random(t.shape) < 0.05).astype(np.uint64) << rng.integers(0, 64, t.shape).astype(np.uint64)
        t[:3] = t[3]  # duplicates: ties in both directions
        for r in (0.0, 0.8, 0.95):
            m, d, ratio, c = ref.match_mutual(q, t, r)
            np.testing.assert_array_equal(m, mutual_by_matrix(q, t, r))
            assert c == int((m >= 0).sum())
            D = distance_matrix(q, t)
            np.testing.assert_array_equal(d, D.min(axis=1))


def test_mutual_recovers_a_permutation(ref):
    rng = np.random.default_rng(71)
    q = rng.integers(0, 2**63, (200, 8), dtype=np.uint64)
    perm = rng.permutation(200)
    t = q[perm]
    m, d, ratio, c = ref.match_mutual(q, t, 0.8)
    assert c == 200
    np.testing.assert_array_equal(perm[m], np.arange(200))
    assert (d == 0).all() and (ratio == 0).all()


def test_mutual_is_symmetric_without_ratio(ref):
    rng = np.random.default_rng(72)
    q = rng.integers(0, 2**63, (80, 2), dtype=np.uint64)
    t = q[:60] ^ (np.uint64(1) << rng.integers(0, 64, (60, 2)).astype(np.uint64))
    t = np.concatenate([t, rng.integers(0, 2**63, (25, 2), dtype=np.uint64)])
    m_qt, *_ = ref.match_mutual(q, t, 0.0)
    m_tq, *_ = ref.match_mutual(t, q, 0.0)
    pairs_qt = {(i, int(j)) for i, j in enumerate(m_qt) if j >= 0}
    pairs_tq = {(int(i), j) for j, i in enumerate(m_tq) if i >= 0}
    assert pairs_qt == pairs_tq and len(pairs_qt) >= 55


def test_ratio_filter_edge_cases(ref):
    q = np.array([[0b1011]], dtype=np.uint64)
    # one train code: no second neighbour, ratio 0, accepted
    m, d, ratio, c = ref.match_mutual(q, np.array([[0b0011]], dtype=np.uint64), 0.5)
    assert m[0] == 0 and d[0] == 1 and ratio[0] == 0.0 and c == 1
    # two equally near train codes: d1 = d2, rejected by any ratio <= 1, kept without the filter
    t = np.array([[0b0011], [0b1001]], dtype=np.uint64)
    m, d, ratio, _ = ref.match_mutual(q, t, 0.99)
    assert m[0] == -1 and ratio[0] == 1.0
    m, _, _, _ = ref.match_mutual(q, t, 0.0)
    assert m[0] == 0
    # d1 = d2 = 0: ratio reported as 1
    _, _, ratio, _ = ref.match_mutual(q, np.array([[0b1011], [0b1011]], dtype=np.uint64), 0.8)
    assert ratio[0] == 1.0
    # 1 < 0.5 * 3 passes, 2 < 0.5 * 3 does not
    t = np.array([[0b1010], [0b0100]], dtype=np.uint64)  # distances 1 and 4
    assert ref.match_mutual(q, t, 0.3)[0][0] == 0
    assert ref.match_mutual(q, t, 0.25)[0][0] == -1  # 1 < 1.0 fails
    # empty train set
    m, d, ratio, c = ref.match_mutual(q, np.zeros((0, 1), dtype=np.uint64), 0.8)
    assert m[0] == -1 and d[0] == 0xFFFFFFFF and c == 0
