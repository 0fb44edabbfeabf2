"""Pins for the oracle's reduced-precision operand rounding (the precision
extension of the projection; the paper fixes no precision).  Rounding is
checked against torch's own bfloat16 and float8_e4m3fn casts (library
routines, round to nearest even); the projection against an FP64 matrix
product of those library-rounded operands."""
import numpy as np
import torch

from paper_2108_08380_amd import synth


def test_bf16_rounding_matches_torch(ref):
    rng = np.random.default_rng(40)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.normal(0, 1e-3, 1000), [0.0, -0.0, 1.0, 1 + 2**-8, 1 + 3 * 2**-8]])
    x = x.astype(np.float32)
    got = np.array([ref.round_bf16(v) for v in x], dtype=np.float32)
    exp = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(got, exp)


def test_e4m3_rounding_matches_torch_in_range(ref):
    rng = np.random.default_rng(41)
    x = np.concatenate([rng.uniform(-448, 448, 3000), rng.normal(0, 0.05, 1000), rng.normal(0, 2**-7, 500),
                        [0.0, 448.0, -448.0, 2**-9, 2**-10, 1.0625, 17.0, 19.0]]).astype(np.float32)
    got = np.array([ref.round_e4m3(v) for v in x], dtype=np.float32)
    exp = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(got, exp)


def test_e4m3_saturates(ref):
    assert ref.round_e4m3(470.0) == 448.0 and ref.round_e4m3(1e6) == 448.0 and ref.round_e4m3(-1e6) == -448.0


def test_project_lowp_matches_library_rounding(ref):
    """BF16 and FP8 operands rounded by torch's own casts; FP8 rows scaled by
    a power of two so that the rescaling itself is exact."""
    rng = np.random.default_rng(42)
    h = rng.random((9, 128)).astype(np.float32)
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    B, t = synth.projection(rng, 256)
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_allclose(ref.project_lowp(h, B, t, "bf16"), bf(h) @ bf(B).T - t.astype(np.float64),
                               rtol=0, atol=1e-12)
    # per-row scale: the smallest power of two s (>= 2^-126) with max|row| <= 448 s, found by search
    def pow2_scale(a):
        out = []
        for m in np.abs(a).max(1).astype(np.float64):
            k = -126
            while m > 448.0 * 2.0 ** k:
                k += 1
            out.append(2.0 ** k)
        return np.array(out, dtype=np.float32)

    sf, sb = pow2_scale(h), pow2_scale(B)
    assert ((np.abs(h).max(1) / sf > 224) & (np.abs(h).max(1) / sf <= 448)).all()
    f8 = lambda a, s: torch.from_numpy((a / s[:, None]).astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    exp = (f8(h, sf) @ f8(B, sb).T) * (sf.astype(np.float64)[:, None] * sb.astype(np.float64)[None, :]) - t
    np.testing.assert_allclose(ref.project_lowp(h, B, t, "fp8"), exp, rtol=0, atol=1e-12)
    # both stay close to the exact projection (error of a few 1e-3 at most for FP8)
    exact = h.astype(np.float64) @ B.astype(np.float64).T - t
    assert np.abs(ref.project_lowp(h, B, t, "bf16") - exact).max() < 5e-3
    assert np.abs(ref.project_lowp(h, B, t, "fp8") - exact).max() < 5e-2
