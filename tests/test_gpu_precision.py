"""Reduced-precision HashSIFT projection (BF16 and FP8-e4m3 MFMA with FP32
accumulation and an FP32 re-check of responses within the margin).

Two parities, as the extension defines them:
  * operand rounding + accumulation: with margin 0 the GPU responses equal
    the FP64 dot products of the same rounded operands (oracle emulation of
    the rounding) up to FP32 accumulation error;
  * against the exact FP64 oracle: the error of responses outside the margin
    and the flipped-bit rate are measured and bounded (BF16) or reported (FP8).
"""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu

MARGIN = 1e-3


def unpack(codes, n_bits):
    return np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")[:, :n_bits]


def features(dev, w, n=None):
    img = torch.from_numpy(w.image1).to(dev)
    kp = w.kp1 if n is None else w.kp1[:n]
    kps = bd.keypoints_tensor(kp, dev)
    return kp, kps, bd.hashsift_features(img, kps)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("n_bits", [256, 512])
def test_rounded_operands_and_accumulation(ref, dev, precision, n_bits):
    w = synth.hashsift512_pair(n_kp=1500, n_bits=n_bits)
    _, kps, f = features(dev, w)
    B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
    _, resp = bd.hashsift_project(f, B, t, kps, precision=precision, with_resp=True, margin=0.0)
    exp = ref.project_lowp(to_np(f), w.B, w.t, precision)
    err = np.abs(to_np(resp) - exp).max()
    print(f"{precision} K={n_bits} max|r_gpu - r_rounded64| = {err:.2e}")
    # A single operand rounded differently from the emulation would move a
    # response by ~1e-3.  BF16 MFMA accumulation matches FP32 rounding (~1e-7);
    # the FP8 instruction's internal sums are coarser (measured up to 2.3e-5).
    assert err <= (2e-5 if precision == "bf16" else 1e-4)


@pytest.mark.parametrize("precision,max_err,max_flip", [("bf16", 5e-3, 1e-4), ("fp8", 6e-2, 5e-2)])
def test_against_fp64_with_recheck(ref, dev, precision, max_err, max_flip):
    w = synth.hashsift512_pair(n_kp=3000)
    kp, kps, f = features(dev, w)
    B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
    count = torch.zeros(1, dtype=torch.uint32, device=dev)
    codes, resp = bd.hashsift_project(f, B, t, kps, precision=precision, with_resp=True, margin=MARGIN,
                                      recheck_count=count)
    _, raw = bd.hashsift_project(f, B, t, kps, precision=precision, with_resp=True, margin=0.0)
    codes, resp, raw, count = to_np(codes), to_np(resp), to_np(raw), int(to_np(count)[0])
    h64, r64, c64 = ref.describe_hashsift(w.image1, kp, w.B, w.t)
    inside = np.abs(raw) < MARGIN
    assert count == int(inside.sum())
    # re-checked responses are FP32 results of the unrounded operands
    assert np.abs(resp[inside] - r64[inside]).max(initial=0) <= 1e-4
    err_out = np.abs(raw[~inside] - r64[~inside]).max()
    flips = (unpack(codes, 512) != unpack(c64, 512)).mean()
    print(f"{precision}: max|r - r64| outside margin {err_out:.2e}, flipped bits {flips:.2e}, "
          f"re-checked {count} of {raw.size} ({count / raw.size:.2e})")
    assert err_out <= max_err
    assert flips <= max_flip


def test_full_size_200k_keypoints(dev):
    """16 images of 1920x1080, 12500 keypoints each (200000): low-precision codes
    against the FP32 path (itself within 4e-7 of FP64)."""
    B = t = None
    stats = {p: [0, 0, 0, 0.0] for p in ("bf16", "fp8")}  # flips, bits, rechecked, max err
    for i in range(16):
        w = synth.hashsift512_pair(synth.SEED_BASE + 3 + 1000 * i, n_kp=12500)
        if B is None:
            B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
        _, kps, f = features(dev, w)
        c32, r32 = bd.hashsift_project(f, B, t, kps, precision="fp32", with_resp=True)
        c32, r32 = to_np(c32), to_np(r32)
        for p in stats:
            cnt = torch.zeros(1, dtype=torch.uint32, device=dev)
            c, r = bd.hashsift_project(f, B, t, kps, precision=p, with_resp=True, margin=MARGIN, recheck_count=cnt)
            c, r = to_np(c), to_np(r)
            s = stats[p]
            s[0] += int((unpack(c, 512) != unpack(c32, 512)).sum())
            s[1] += c.size * 64
            s[2] += int(to_np(cnt)[0])
            s[3] = max(s[3], float(np.abs(r - r32).max()))
    for p, (fl, nb, rc, e) in stats.items():
        print(f"{p}: flipped {fl}/{nb} = {fl / nb:.2e}, re-checked {rc} ({rc / nb:.2e}), max|r - r32| {e:.2e}")
    assert stats["bf16"][0] / stats["bf16"][1] <= 1e-4
    assert stats["fp8"][0] / stats["fp8"][1] <= 5e-2


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("n_bits", [256, 512])
def test_margin_covering_every_response(dev, precision, n_bits):
    """margin 10: every response is re-checked from the unrounded FP32
    operands, so each code bit is the sign of the exact response (FP32 sum,
    FP64 within 1e-6 of the threshold) and every response is counted.  The
    per-wavefront list of pending lanes fills and is re-checked part-way
    through each tile."""
    w = synth.hashsift512_pair(n_kp=700, n_bits=n_bits)
    _, kps, f = features(dev, w)
    B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
    count = torch.zeros(1, dtype=torch.uint32, device=dev)
    codes, resp = bd.hashsift_project(f, B, t, kps, precision=precision, with_resp=True, margin=10.0,
                                      recheck_count=count)
    exact = to_np(f).astype(np.float64) @ w.B.astype(np.float64).T - w.t.astype(np.float64)
    assert int(to_np(count)[0]) == exact.size
    assert np.abs(to_np(resp) - exact).max() <= 2e-6
    assert (unpack(to_np(codes), n_bits) == (exact > 0)).all()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_nan_rows_zero_rows_and_signed_zero_thresholds(ref, dev, precision):
    """Without a margin the code bit is r > 0 from the rounded operands:
    a row of NaN gives zero bits, a zero row against thresholds +0 and -0
    gives r = +0 (bit 0), and a row scaled by 2^70 (beyond the range where
    the sign is read without a check) keeps the signs of the emulation."""
    rng = np.random.default_rng(2108)
    n = 203
    f = rng.random((n, 128)).astype(np.float32)
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    B = rng.normal(0.0, 1.0 / np.sqrt(128.0), (512, 128)).astype(np.float32)
    t = rng.normal(0.0, 0.01, 512).astype(np.float32)
    t[0::3] = -0.0
    t[1::3] = 0.0
    f[3] = 0.0
    f[4] = np.nan
    f[130] *= np.float32(2.0 ** 70)
    codes, resp = bd.hashsift_project(torch.from_numpy(f).to(dev), torch.from_numpy(B).to(dev),
                                      torch.from_numpy(t).to(dev), precision=precision, with_resp=True, margin=0.0)
    bits = unpack(to_np(codes), 512)
    emul = ref.project_lowp(np.nan_to_num(f, nan=0.0), B, t, precision)
    assert not bits[4].any()
    assert (bits[3] == (-t.astype(np.float64) > 0)).all()
    assert not bits[3][0::3].any() and not bits[3][1::3].any()
    rows = [i for i in range(n) if i != 4]
    clear = np.abs(emul[rows]) > np.abs(emul[rows]).max(axis=1, keepdims=True) * 1e-3
    assert (bits[rows] == (emul[rows] > 0))[clear].all()


@pytest.mark.parametrize("margin", [0.0, 1e-3])
def test_fp8_extreme_row_scales(ref, dev, margin):
    """FP8 rows of B (and their thresholds) scaled by 2^-70 and 2^40, so row
    scales of one chunk differ by up to 2^110: bits match the emulation of
    the same rounding wherever the response is clear of zero, and with a
    margin the re-check decides the rest."""
    rng = np.random.default_rng(70)
    n = 333
    f = rng.random((n, 128)).astype(np.float32)
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    B = rng.normal(0.0, 1.0 / np.sqrt(128.0), (512, 128)).astype(np.float32)
    t = rng.normal(0.0, 0.01, 512).astype(np.float32)
    B[5:9] *= np.float32(2.0 ** -70)
    t[5:9] *= np.float32(2.0 ** -70)
    B[300:303] *= np.float32(2.0 ** 40)
    t[300:303] *= np.float32(2.0 ** 40)
    codes, resp = bd.hashsift_project(torch.from_numpy(f).to(dev), torch.from_numpy(B).to(dev),
                                      torch.from_numpy(t).to(dev), precision="fp8", with_resp=True, margin=margin)
    bits = unpack(to_np(codes), 512)
    emul = ref.project_lowp(f, B, t, "fp8")
    scale = np.abs(emul).max(axis=0, keepdims=True)  # per bit: rows of B differ by 2^110
    # the FP8 rounding moves a response by a few per cent of its bit's scale
    clear = np.abs(emul) > 0.2 * scale
    assert (bits == (emul > 0))[clear].all()
    assert (np.abs(to_np(resp) - emul) / scale).max() <= 0.15
    if margin == 0.0:
        # without a re-check every bit is the sign of the emulated response, up to FP32 accumulation
        assert (bits == (emul > 0))[np.abs(emul) > 1e-4 * scale].all()
