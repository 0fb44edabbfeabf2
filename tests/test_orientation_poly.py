"""The HashSIFT kernel's orientation polynomial (csrc/hashsift.hip,
orientation_bin), evaluated on the CPU in float32 exactly as the kernel's
operations round, against numpy's arctan2 on dense grids.  Pins:
  * its constants are the fit of paper_2108_08380_amd/fit_orientation.py
    rounded to float32;
  * the polynomial itself (evaluated in float64) is within 1.2e-7 bins of
    atan(t) * 4/pi on the first octant;
  * the float32 evaluation on the octant is within 2.4e-7 bins;
  * the full bin coordinate in [0, 8] is within 5.5e-7 bins of
    atan2(gy, gx) * 8/(2 pi) at every angle and magnitude tried (half an
    ulp of 8, 2.4e-7, comes from storing values near 8 in float32)."""
import os
import re

import numpy as np

from paper_2108_08380_amd import fit_orientation

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
f32 = np.float32


def kernel_coefficients():
    src = open(os.path.join(ROOT, "paper_2108_08380_amd", "csrc", "hashsift.hip")).read()
    body = src[src.index("orientation_bin(float gx, float gy)"):]
    body = body[:body.index("return b;")]
    first = re.search(r"float p = (-?[0-9.eE+-]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, u, (-?[0-9.eE+-]+)f\);", body)
    return np.array([first, *rest], dtype=np.float64)


def fma32(a, b, c):
    # a*b of two float32 values is exact in float64; one rounding of the sum
    # to float64 then to float32 equals the fused result except in ties
    # far below the bounds pinned here
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def octant(t, coef):
    u = (t * t).astype(f32)
    p = np.full_like(u, f32(coef[0]))
    for c in coef[1:]:
        p = fma32(p, u, np.full_like(u, f32(c)))
    return (t * p).astype(f32)


def bin_coordinate(gx, gy, coef):
    ax, ay = np.abs(gx), np.abs(gy)
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    # the kernel's reciprocal is the hardware's (1 ulp); a correctly rounded one here
    r = (1.0 / np.maximum(mx, f32(1e-30)).astype(np.float64)).astype(f32)
    b = octant((mn * r).astype(f32), coef)
    b = np.where(ay > ax, f32(2) - b, b).astype(f32)
    b = np.where(gx < 0, f32(4) - b, b).astype(f32)
    return np.where(gy < 0, f32(8) - b, b).astype(f32)


def test_constants_are_the_committed_fit():
    coef = kernel_coefficients()
    assert len(coef) == fit_orientation.DEGREE + 1
    np.testing.assert_array_equal(coef.astype(f32), fit_orientation.fit().astype(f32))


def test_octant_error():
    coef = kernel_coefficients()
    t = np.linspace(0.0, 1.0, 2_000_001).astype(f32)
    exact = np.arctan(t.astype(np.float64)) * 4.0 / np.pi
    poly = t.astype(np.float64) * np.polyval(coef, t.astype(np.float64) ** 2)
    assert np.abs(poly - exact).max() <= 1.2e-7
    assert np.abs(octant(t, coef).astype(np.float64) - exact).max() <= 2.4e-7
    assert octant(np.array([0.0], f32), coef)[0] == 0.0


def test_full_circle_error_and_special_directions():
    coef = kernel_coefficients()
    ang = np.linspace(0.0, 2.0 * np.pi, 1_000_003, endpoint=False)
    for mag in (1e-3, 0.37, 1.0, 255.0, 3.1e4):
        gx = (mag * np.cos(ang)).astype(f32)
        gy = (mag * np.sin(ang)).astype(f32)
        b = bin_coordinate(gx, gy, coef).astype(np.float64)
        exact = np.mod(np.arctan2(gy.astype(np.float64), gx.astype(np.float64)), 2.0 * np.pi) * 8.0 / (2.0 * np.pi)
        d = np.abs(b - exact)
        assert np.minimum(d, 8.0 - d).max() <= 5.5e-7, mag
        assert ((b >= 0.0) & (b <= 8.0)).all()
    # axes and diagonals land on their bins exactly (up to the polynomial at t = 1)
    gx = np.array([1, 0, -1, 0, 0], f32)
    gy = np.array([0, 1, 0, -1, 0], f32)
    np.testing.assert_array_equal(bin_coordinate(gx, gy, coef), np.array([0, 2, 4, 6, 0], f32))
    diag = bin_coordinate(np.array([1, -1, -1, 1], f32), np.array([1, 1, -1, -1], f32), coef)
    np.testing.assert_allclose(diag, [1, 3, 5, 7], atol=2.4e-7)
