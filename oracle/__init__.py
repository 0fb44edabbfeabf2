"""Python access to the CPU oracle (bdref.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the library.  The oracle shares no
code with the GPU path; this module only marshals numpy arrays into the C
functions declared in bdref.h.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bdref.c")
_LIB_PATH = os.path.join(_HERE, "libbdref.so")

KEYPOINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("scale", "<f4"), ("angle", "<f4")])
BOX_PAIR_DTYPE = np.dtype([("x1", "i1"), ("y1", "i1"), ("x2", "i1"), ("y2", "i1"),
                           ("radius", "u1"), ("pad", "u1", (3,)), ("threshold", "<f4")])


def build() -> str:
    """Compile bdref.c with plain IEEE FP64 semantics (no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.bdref_build_integral.argtypes = [P, i32, i32, i64, P, i64]
        L.bdref_build_integral.restype = None
        L.bdref_describe_bad.argtypes = [P, i32, i32, i64, P, i32, P, i32, P]
        L.bdref_describe_bad.restype = i64
        L.bdref_hashsift_hist.argtypes = [P, i32, i32, i32, i64, P, i32, P]
        L.bdref_hashsift_hist.restype = None
        L.bdref_hashsift_project.argtypes = [P, i32, P, P, i32, P, P, P]
        L.bdref_hashsift_project.restype = None
        L.bdref_keypoint_valid.argtypes = [P]
        L.bdref_keypoint_valid.restype = i32
        L.bdref_match_knn.argtypes = [P, i32, P, i32, i32, i32, P, P]
        L.bdref_match_knn.restype = None
        L.bdref_match_mutual.argtypes = [P, i32, P, i32, i32, ctypes.c_double, P, P, P]
        L.bdref_match_mutual.restype = i32
        L.bdref_threshold_bin.argtypes = [P, P]
        L.bdref_threshold_bin.restype = i32
        L.bdref_find_threshold.argtypes = [P, i32, P, P, ctypes.c_double, P, i32, P, P]
        L.bdref_find_threshold.restype = None
        L.bdref_hnm_codes.argtypes = [P, P, i32, i32, P, P, P]
        L.bdref_hnm_codes.restype = None
        L.bdref_select_features.argtypes = [P, i32, P, i32, P, i32, i32, ctypes.c_double, P, P, P, P, P]
        L.bdref_select_features.restype = None
        L.bdref_augment_patches.argtypes = [P, i32, P, P, P]
        L.bdref_augment_patches.restype = None
        L.bdref_round_bf16.argtypes = [ctypes.c_float]
        L.bdref_round_bf16.restype = ctypes.c_float
        L.bdref_round_e4m3.argtypes = [ctypes.c_float]
        L.bdref_round_e4m3.restype = ctypes.c_float
        L.bdref_project_lowp.argtypes = [P, i32, P, P, i32, i32, P]
        L.bdref_project_lowp.restype = None
        d = ctypes.c_double
        L.bdref_relaxed_bad.argtypes = [P, i32, P, P, P, P, i32, d, P, P, P, P]
        L.bdref_relaxed_bad.restype = None
        L.bdref_relaxed_hashsift.argtypes = [P, i32, P, P, i32, d, P, P]
        L.bdref_relaxed_hashsift.restype = None
        L.bdref_trl_hnm.argtypes = [P, P, i32, i32, d, P, P, P]
        L.bdref_trl_hnm.restype = d
        L.bdref_relaxed_bad_grad.argtypes = [P, P, P, P, i32, i32, d, P, P, P]
        L.bdref_relaxed_bad_grad.restype = None
        L.bdref_relaxed_hashsift_grad.argtypes = [P, P, P, i32, i32, d, P, P]
        L.bdref_relaxed_hashsift_grad.restype = None
        L.bdref_hashsift_patch_features.argtypes = [P, i32, P]
        L.bdref_hashsift_patch_features.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _as_keypoints(kp) -> np.ndarray:
    kp = np.ascontiguousarray(kp)
    if kp.dtype != KEYPOINT_DTYPE:
        kp = np.ascontiguousarray(np.asarray(kp, dtype=np.float32).reshape(-1, 4)).view(KEYPOINT_DTYPE).reshape(-1)
    return kp


def _as_pairs(pairs) -> np.ndarray:
    pairs = np.ascontiguousarray(pairs)
    assert pairs.dtype.itemsize == 12
    return pairs


def build_integral(img: np.ndarray) -> np.ndarray:
    """(H, W) u8 -> (H+1, W+1) u32 integral image."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    ii = np.empty((H + 1, W + 1), dtype=np.uint32)
    lib().bdref_build_integral(_ptr(img), W, H, W, _ptr(ii), W + 1)
    return ii


def describe_bad(ii: np.ndarray, kps, pairs, n_bits: int | None = None):
    """BAD codes from an integral image.  Returns (codes (n, n_bits/64) u64, near_tie_count)."""
    ii = np.ascontiguousarray(ii, dtype=np.uint32)
    kp = _as_keypoints(kps)
    pr = _as_pairs(pairs)
    n_bits = len(pr) if n_bits is None else n_bits
    assert n_bits % 64 == 0 and len(pr) >= n_bits
    H, W = ii.shape[0] - 1, ii.shape[1] - 1
    codes = np.zeros((len(kp), n_bits // 64), dtype=np.uint64)
    ties = lib().bdref_describe_bad(_ptr(ii), W, H, ii.shape[1], _ptr(kp), len(kp), _ptr(pr),
                                    n_bits, _ptr(codes))
    return codes, int(ties)


def hashsift_hist(img: np.ndarray, kps) -> np.ndarray:
    """(n, 128) FP64 L2-normalized 4x4x8 histograms; img is u8 or f32 (H, W)."""
    img = np.ascontiguousarray(img)
    if img.dtype == np.uint8:
        dtype = 0
    elif img.dtype == np.float32:
        dtype = 1
    else:
        raise TypeError("image must be uint8 or float32")
    kp = _as_keypoints(kps)
    H, W = img.shape
    hist = np.zeros((len(kp), 128), dtype=np.float64)
    lib().bdref_hashsift_hist(_ptr(img), dtype, W, H, img.strides[0], _ptr(kp), len(kp), _ptr(hist))
    return hist


def keypoint_valid(kps) -> np.ndarray:
    kp = _as_keypoints(kps)
    L = lib()
    return np.array([L.bdref_keypoint_valid(_ptr(kp[i:i + 1])) for i in range(len(kp))], dtype=np.uint8)


def hashsift_project(hist: np.ndarray, B: np.ndarray, t: np.ndarray, valid=None):
    """Responses r = B f - t (FP64) and codes (bit set when r > 0)."""
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    n_bits = B.shape[0]
    assert B.shape[1] == 128 and t.shape == (n_bits,) and n_bits % 64 == 0
    n = hist.shape[0]
    resp = np.zeros((n, n_bits), dtype=np.float64)
    codes = np.zeros((n, n_bits // 64), dtype=np.uint64)
    vptr = None
    if valid is not None:
        valid = np.ascontiguousarray(valid, dtype=np.uint8)
        vptr = _ptr(valid)
    lib().bdref_hashsift_project(_ptr(hist), n, _ptr(B), _ptr(t), n_bits, vptr, _ptr(resp), _ptr(codes))
    return resp, codes


def describe_hashsift(img: np.ndarray, kps, B: np.ndarray, t: np.ndarray):
    """Histogram, responses and codes of the HashSIFT descriptor."""
    hist = hashsift_hist(img, kps)
    resp, codes = hashsift_project(hist, B, t, keypoint_valid(kps))
    return hist, resp, codes


def match_knn(query: np.ndarray, train: np.ndarray, k: int):
    """Brute-force Hamming k-NN; returns (idx (n_q, k) i32, dist (n_q, k) u32)."""
    q = np.ascontiguousarray(query, dtype=np.uint64)
    t = np.ascontiguousarray(train, dtype=np.uint64)
    n_words = q.shape[1]
    assert t.shape[1] == n_words
    idx = np.empty((q.shape[0], k), dtype=np.int32)
    dist = np.empty((q.shape[0], k), dtype=np.uint32)
    lib().bdref_match_knn(_ptr(q), q.shape[0], _ptr(t), t.shape[0], n_words, k, _ptr(idx), _ptr(dist))
    return idx, dist


def match_mutual(query: np.ndarray, train: np.ndarray, max_ratio: float = 0.0):
    """Mutual nearest neighbours with the distance-ratio filter.
    Returns (match (n_q,) i32, dist (n_q,) u32, ratio (n_q,) f64, count)."""
    q = np.ascontiguousarray(query, dtype=np.uint64)
    t = np.ascontiguousarray(train, dtype=np.uint64)
    n_words = q.shape[1]
    assert t.shape[1] == n_words
    match = np.empty(q.shape[0], dtype=np.int32)
    dist = np.empty(q.shape[0], dtype=np.uint32)
    ratio = np.empty(q.shape[0], dtype=np.float64)
    count = lib().bdref_match_mutual(_ptr(q), q.shape[0], _ptr(t), t.shape[0], n_words, float(max_ratio),
                                     _ptr(match), _ptr(dist), _ptr(ratio))
    return match, dist, ratio, int(count)


PRECISIONS = {"bf16": 1, "fp8": 2}


def round_bf16(x: float) -> float:
    return float(lib().bdref_round_bf16(float(x)))


def round_e4m3(x: float) -> float:
    return float(lib().bdref_round_e4m3(float(x)))


def project_lowp(hist32: np.ndarray, B: np.ndarray, t: np.ndarray, precision: str) -> np.ndarray:
    """FP64 responses of the projection with BF16- or FP8-rounded operands."""
    h = np.ascontiguousarray(hist32, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    resp = np.zeros((h.shape[0], B.shape[0]), dtype=np.float64)
    lib().bdref_project_lowp(_ptr(h), h.shape[0], _ptr(B), _ptr(t), B.shape[0], PRECISIONS[precision], _ptr(resp))
    return resp


# --------------------------------------------------------------------------- differentiation


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def relaxed_bad(patches, pairs, w1, w2, theta, beta):
    """(rho, D, m1, m2), each (n, K) FP64."""
    pt = np.ascontiguousarray(patches, dtype=np.float32).reshape(-1, 1024)
    pr = _as_pairs(pairs)
    n, K = pt.shape[0], len(pr)
    w1, w2, theta = _f64(w1), _f64(w2), _f64(theta)
    out = [np.zeros((n, K)) for _ in range(4)]
    lib().bdref_relaxed_bad(_ptr(pt), n, _ptr(pr), _ptr(w1), _ptr(w2), _ptr(theta), K, float(beta),
                            *[_ptr(o) for o in out])
    return tuple(out)


def relaxed_hashsift(f, B, t, beta):
    """(rho, D), each (n, K) FP64, for features f (n, 128)."""
    f, B, t = _f64(f), _f64(B), _f64(t)
    n, K = f.shape[0], B.shape[0]
    rho, dt = np.zeros((n, K)), np.zeros((n, K))
    lib().bdref_relaxed_hashsift(_ptr(f), n, _ptr(B), _ptr(t), K, float(beta), _ptr(rho), _ptr(dt))
    return rho, dt


def trl_hnm(A, P, tau, grads=True):
    """(loss, neg, gA, gP) of the in-batch hardest-negative triplet ranking loss."""
    A, P = _f64(A), _f64(P)
    n, K = A.shape
    neg = np.zeros(n, dtype=np.int32)
    gA, gP = (np.zeros((n, K)), np.zeros((n, K))) if grads else (None, None)
    loss = lib().bdref_trl_hnm(_ptr(A), _ptr(P), n, K, float(tau), _ptr(neg),
                               _ptr(gA) if grads else None, _ptr(gP) if grads else None)
    return loss, neg, gA, gP


def relaxed_bad_grad(gD, dt, m1, m2, beta):
    gD, dt, m1, m2 = _f64(gD), _f64(dt), _f64(m1), _f64(m2)
    n, K = gD.shape
    g = [np.zeros(K) for _ in range(3)]
    lib().bdref_relaxed_bad_grad(_ptr(gD), _ptr(dt), _ptr(m1), _ptr(m2), n, K, float(beta), *[_ptr(x) for x in g])
    return tuple(g)  # (g_w1, g_w2, g_theta)


def relaxed_hashsift_grad(gD, dt, f, beta):
    gD, dt, f = _f64(gD), _f64(dt), _f64(f)
    n, K = gD.shape
    gB, gt = np.zeros((K, 128)), np.zeros(K)
    lib().bdref_relaxed_hashsift_grad(_ptr(gD), _ptr(dt), _ptr(f), n, K, float(beta), _ptr(gB), _ptr(gt))
    return gB, gt


def hashsift_patch_features(patches):
    pt = np.ascontiguousarray(patches, dtype=np.float32).reshape(-1, 1024)
    f = np.zeros((pt.shape[0], 128))
    lib().bdref_hashsift_patch_features(_ptr(pt), pt.shape[0], _ptr(f))
    return f


THRESHOLD_BINS = 5110


def threshold_bin(patch: np.ndarray, cand) -> int:
    """Bin q = floor((f + 255) * 10) of one candidate feature on one u8 32x32 patch."""
    p = np.ascontiguousarray(patch, dtype=np.uint8).reshape(32, 32)
    c = _as_pairs(np.atleast_1d(cand))
    return int(lib().bdref_threshold_bin(_ptr(p), _ptr(c)))


def find_threshold(patches: np.ndarray, s_ap, s_an, tau: float, cands):
    """Alg. 2 for each candidate over the triplets (patches (3n, 32, 32) u8, a/p/n
    interleaved).  Returns (best_bin (J,) int32, best_loss (J,) float64)."""
    p = np.ascontiguousarray(patches, dtype=np.uint8)
    n = p.shape[0] // 3
    assert p.shape[0] == 3 * n and p[0].size == 1024
    sap = np.ascontiguousarray(s_ap, dtype=np.int32)
    san = np.ascontiguousarray(s_an, dtype=np.int32)
    assert sap.shape == (n,) and san.shape == (n,)
    c = _as_pairs(cands)
    best_bin = np.empty(len(c), dtype=np.int32)
    best_loss = np.empty(len(c), dtype=np.float64)
    lib().bdref_find_threshold(_ptr(p), n, _ptr(sap), _ptr(san), float(tau), _ptr(c), len(c), _ptr(best_bin),
                               _ptr(best_loss))
    return best_bin, best_loss


def hnm_codes(a_codes: np.ndarray, p_codes: np.ndarray):
    """In-batch hardest negatives with anchor swap.  Returns (neg, dist_neg, dist_pos), int32 (n,)."""
    a = np.ascontiguousarray(a_codes, dtype=np.uint64)
    p = np.ascontiguousarray(p_codes, dtype=np.uint64)
    n, w = a.shape
    neg = np.empty(n, np.int32)
    dn = np.empty(n, np.int32)
    dp = np.empty(n, np.int32)
    lib().bdref_hnm_codes(_ptr(a), _ptr(p), n, w, _ptr(neg), _ptr(dn), _ptr(dp))
    return neg, dn, dp


def select_features(pool: np.ndarray, samples: np.ndarray, cands: np.ndarray, tau: float):
    """Alg. 1: pool (2P, 32, 32) u8 (anchor, positive interleaved), samples (K, N) int32 pair
    indices, cands (K, J) box pairs.  Returns (table (K,) box pairs, chosen (K,), chosen_bin (K,),
    round_loss (K,), pool_codes (2P, ceil(K/64)) u64)."""
    pl = np.ascontiguousarray(pool, dtype=np.uint8)
    n_pairs = pl.shape[0] // 2
    smp = np.ascontiguousarray(samples, dtype=np.int32)
    K, N = smp.shape
    c = _as_pairs(cands)
    assert c.shape[0] == K
    J = c.shape[1]
    table = np.zeros(K, dtype=c.dtype)
    chosen = np.empty(K, np.int32)
    chosen_bin = np.empty(K, np.int32)
    loss = np.empty(K, np.float64)
    codes = np.zeros((2 * n_pairs, (K + 63) // 64), np.uint64)
    lib().bdref_select_features(_ptr(pl), n_pairs, _ptr(smp), N, _ptr(c), J, K, float(tau), _ptr(table),
                                _ptr(chosen), _ptr(chosen_bin), _ptr(loss), _ptr(codes))
    return table, chosen, chosen_bin, loss, codes


# ---------------------------------------------------------------- HashSIFT training (Sec. III-B)


def augment_patches(src: np.ndarray, params: np.ndarray, noise: np.ndarray) -> np.ndarray:
    """Rotation/scale, blur, illumination and noise of (n, 32, 32) float patches;
    params (n, 5) = (angle, scale, gain, bias, sigma), noise (n, 32, 32)."""
    sp = np.ascontiguousarray(src, dtype=np.float32).reshape(-1, 1024)
    n = sp.shape[0]
    pr = np.ascontiguousarray(params, dtype=np.float64).reshape(n, 5)
    nz = np.ascontiguousarray(noise, dtype=np.float32).reshape(n, 1024)
    out = np.empty((n, 1024), dtype=np.float32)
    lib().bdref_augment_patches(_ptr(sp), n, _ptr(pr), _ptr(nz), _ptr(out))
    return out.reshape(n, 32, 32)


def adam_step(param, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba) of FP64 arrays, in place; step counts from 1."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    param -= lr * m_hat / (np.sqrt(v_hat) + eps)


def hashsift_train_step(pool, batch, params, noise, B, t, state, lr=2e-4, tau=0.5, beta=1.0,
                        beta1=0.9, beta2=0.999, eps=1e-8):
    """One training iteration of the HashSIFT projection (Sec. III-B, Eq. 3):
    pair s of the batch is pool pair batch[s] (anchor 2 batch[s], positive
    2 batch[s] + 1), augmented with params / noise rows 2s (anchor) and 2s + 1
    (positive); relaxed descriptors tanh(beta (B f - t)); triplet loss with
    in-batch hardest negatives and anchor swap; Adam on B and t.  B, t and
    state = {"mB", "vB", "mt", "vt", "step"} are updated in place.  Returns
    (loss, gB, gt)."""
    pool = np.asarray(pool).reshape(-1, 32, 32)
    idx = np.asarray(batch, dtype=np.int64)
    n = len(idx)
    src = np.empty((2 * n, 32, 32), dtype=np.float32)
    src[0::2], src[1::2] = pool[2 * idx], pool[2 * idx + 1]
    aug = augment_patches(src, params, noise)
    fa, fp = hashsift_patch_features(aug[0::2]), hashsift_patch_features(aug[1::2])
    _, Da = relaxed_hashsift(fa, B, t, beta)
    _, Dp = relaxed_hashsift(fp, B, t, beta)
    loss, _, gA, gP = trl_hnm(Da, Dp, tau)
    gBa, gta = relaxed_hashsift_grad(gA, Da, fa, beta)
    gBp, gtp = relaxed_hashsift_grad(gP, Dp, fp, beta)
    gB, gt = gBa + gBp, gta + gtp
    state["step"] += 1
    adam_step(B, gB, state["mB"], state["vB"], state["step"], lr, beta1, beta2, eps)
    adam_step(t, gt, state["mt"], state["vt"], state["step"], lr, beta1, beta2, eps)
    return loss, gB, gt
