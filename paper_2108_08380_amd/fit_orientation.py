"""Coefficients of the orientation polynomial in csrc/hashsift.hip.

The HashSIFT histogram needs each gradient's angle as a bin coordinate
atan2(gy, gx) * 8 / (2 pi) (Sec. III-B: SIFT-style 8-orientation votes).
The kernel reduces the angle to the first octant, t = min/max in [0, 1],
and evaluates atan(t) * 4/pi as t * P(t^2) with P of degree 7.  P is fitted
here: least squares of t * P(u) against atan(t) * 4/pi on 2000 Chebyshev
nodes of u = t^2 in [0, 1], reweighted 200 times by the current absolute
error (Lawson's iteration towards the minimax fit).  The kernel's constants
are these values rounded to float32.

`python -m paper_2108_08380_amd.fit_orientation` prints them, highest power
first (the order of the kernel's Horner steps)."""
from __future__ import annotations

import numpy as np

DEGREE = 7
NODES = 2000
ITERATIONS = 200


def fit() -> np.ndarray:
    """float64 coefficients, highest power of u first."""
    k = np.arange(NODES)
    u = 0.5 - 0.5 * np.cos((2 * k + 1) * np.pi / (2 * NODES))
    t = np.sqrt(u)
    target = np.arctan(t) * 4.0 / np.pi
    V = np.stack([t * u ** j for j in range(DEGREE + 1)], axis=1)
    w = np.ones(NODES)
    for _ in range(ITERATIONS):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], target * sw, rcond=None)
        err = np.abs(V @ c - target)
        w = w * err
        w /= w.sum()
    return c[::-1].copy()


if __name__ == "__main__":
    for v in fit().astype(np.float32):
        print(repr(float(v)))
