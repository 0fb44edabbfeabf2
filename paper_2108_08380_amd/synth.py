"""Seeded synthetic workloads with the shapes of the paper's inputs.

The paper times description on the Oxford images (about 800 px wide, at most
2000 keypoints per image; Sec. IV, execution-time experiment) and trains on
32x32 patch triplets from the Brown/HPatches sets (Sec. III-A).  None of those
datasets is used: these generators produce seeded stand-ins of the same shape.

This module is input generation only.  It holds none of the arithmetic of the
descriptors or of the matcher, so both the GPU path and the CPU oracle can be
fed from it.  Every draw comes from numpy's PCG64 with independent streams
spawned from one seed per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 210808380

# Keypoint record as the library reads it: image-pixel centre (x right, y
# down, pixel centres on integers), scale = image pixels per normalized-patch
# pixel, angle in radians.
KEYPOINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("scale", "<f4"), ("angle", "<f4")])

# One BAD weak descriptor: two box centres as integer offsets from the
# keypoint in normalized-patch pixels, a box radius (box side 2r+1 before
# scaling) and a threshold in grey levels.  12 bytes, little-endian.
BOX_PAIR_DTYPE = np.dtype(
    [
        ("x1", "i1"),
        ("y1", "i1"),
        ("x2", "i1"),
        ("y2", "i1"),
        ("radius", "u1"),
        ("pad", "u1", (3,)),
        ("threshold", "<f4"),
    ]
)
assert KEYPOINT_DTYPE.itemsize == 16 and BOX_PAIR_DTYPE.itemsize == 12


def streams(seed: int, n: int = 6) -> list[np.random.Generator]:
    """Independent generators spawned from one seed (image, keypoints, params, noise, ...)."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


# --------------------------------------------------------------------------- images


def _smoothstep_axis(n: int, cell: int) -> tuple[np.ndarray, np.ndarray]:
    pos = np.arange(n, dtype=np.float64) / cell
    i0 = np.floor(pos).astype(np.int64)
    f = pos - i0
    return i0, f * f * (3.0 - 2.0 * f)


def value_noise(rng: np.random.Generator, height: int, width: int,
                octaves=((64, 1.0), (32, 0.5), (16, 0.25), (8, 0.125))) -> np.ndarray:
    """Smooth value noise in [0, 255] (float64): random lattice values, smoothstep blend."""
    img = np.zeros((height, width), dtype=np.float64)
    for cell, amp in octaves:
        lat = rng.random((height // cell + 2, width // cell + 2))
        iy, sy = _smoothstep_axis(height, cell)
        ix, sx = _smoothstep_axis(width, cell)
        # blend along x on the lattice rows first, then gather rows and blend along y
        lat_x = lat[:, ix] * (1.0 - sx) + lat[:, ix + 1] * sx
        img += amp * (lat_x[iy] * (1.0 - sy)[:, None] + lat_x[iy + 1] * sy[:, None])
    lo, hi = img.min(), img.max()
    return (img - lo) * (255.0 / max(hi - lo, 1e-12))


def paint_rectangles(rng: np.random.Generator, img: np.ndarray, count: int) -> None:
    """Paint `count` filled axis-aligned rectangles in order (grey level 0..255)."""
    h, w = img.shape
    side_max = max(8, min(w, h) // 4)
    for _ in range(count):
        rw = int(rng.integers(8, side_max + 1))
        rh = int(rng.integers(8, side_max + 1))
        x0 = int(rng.integers(0, max(1, w - rw + 1)))
        y0 = int(rng.integers(0, max(1, h - rh + 1)))
        img[y0:y0 + rh, x0:x0 + rw] = float(rng.integers(0, 256))


def rectangle_count(width: int, height: int) -> int:
    """50 rectangles on 640x480, scaled with the image area."""
    return int(round(50.0 * width * height / (640 * 480)))


def grey_image(rng: np.random.Generator, width: int, height: int,
               n_rect: int | None = None) -> np.ndarray:
    """Float64 grey image in [0, 255]: value noise plus filled rectangles."""
    img = value_noise(rng, height, width)
    paint_rectangles(rng, img, rectangle_count(width, height) if n_rect is None else n_rect)
    return img


def quantize_u8(img: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def shifted_noisy_copy(rng: np.random.Generator, img: np.ndarray, dx: int = 3, dy: int = 2,
                       noise_sigma: float = 4.0, scale: float = 255.0) -> np.ndarray:
    """Second view: content moved by (dx, dy) px (edge replicated) plus Gaussian noise.

    `img` is u8 (noise in grey levels, rounded and clipped) or float in [0, 1]
    (noise sigma divided by `scale`, clipped to [0, 1])."""
    h, w = img.shape
    ys = np.clip(np.arange(h) - dy, 0, h - 1)
    xs = np.clip(np.arange(w) - dx, 0, w - 1)
    moved = img[ys][:, xs].astype(np.float64)
    if img.dtype == np.uint8:
        return quantize_u8(moved + rng.normal(0.0, noise_sigma, size=moved.shape))
    out = moved + rng.normal(0.0, noise_sigma / scale, size=moved.shape)
    return np.clip(out, 0.0, 1.0).astype(img.dtype)


# --------------------------------------------------------------------------- keypoints / parameters


def keypoints(rng: np.random.Generator, n: int, width: int, height: int, border: float = 32.0,
              scale_range=(1.0, 4.0)) -> np.ndarray:
    kp = np.empty(n, dtype=KEYPOINT_DTYPE)
    kp["x"] = rng.uniform(border, width - border, n)
    kp["y"] = rng.uniform(border, height - border, n)
    kp["scale"] = rng.uniform(scale_range[0], scale_range[1], n)
    kp["angle"] = rng.uniform(0.0, 2.0 * math.pi, n)
    return kp


def shift_keypoints(kp: np.ndarray, dx: float, dy: float) -> np.ndarray:
    out = kp.copy()
    out["x"] += np.float32(dx)
    out["y"] += np.float32(dy)
    return out


def box_pairs(rng: np.random.Generator, n_bits: int, max_offset: int = 14,
              radius_range=(1, 5), threshold_range=(-20, 20)) -> np.ndarray:
    """Random BAD table: offsets U{-14..14}^2, radius U{1..5}, integer thresholds U{-20..20}."""
    p = np.zeros(n_bits, dtype=BOX_PAIR_DTYPE)
    for name in ("x1", "y1", "x2", "y2"):
        p[name] = rng.integers(-max_offset, max_offset + 1, n_bits)
    p["radius"] = rng.integers(radius_range[0], radius_range[1] + 1, n_bits)
    p["threshold"] = rng.integers(threshold_range[0], threshold_range[1] + 1, n_bits).astype(np.float32)
    return p


def projection(rng: np.random.Generator, n_bits: int, dim: int = 128,
               b_var: float = 1.0 / 128.0, t_var: float = 0.01) -> tuple[np.ndarray, np.ndarray]:
    """HashSIFT parameters: B (n_bits x dim) ~ N(0, b_var), thresholds t ~ N(0, t_var) (variances)."""
    B = rng.normal(0.0, math.sqrt(b_var), (n_bits, dim)).astype(np.float32)
    t = rng.normal(0.0, math.sqrt(t_var), n_bits).astype(np.float32)
    return B, t


def random_codes(rng: np.random.Generator, n: int, n_words: int) -> np.ndarray:
    return rng.integers(0, 2**64, size=(n, n_words), dtype=np.uint64, endpoint=False)


# --------------------------------------------------------------------------- named workloads


@dataclass
class ImagePairWorkload:
    """Two views of one synthetic scene plus keypoints and descriptor parameters."""

    name: str
    image1: np.ndarray
    image2: np.ndarray
    kp1: np.ndarray
    kp2: np.ndarray
    pairs: np.ndarray | None = None
    B: np.ndarray | None = None
    t: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def bad256_pair(seed: int = SEED_BASE + 0, width: int = 640, height: int = 480, n_kp: int = 1000,
                n_bits: int = 256, scale_range=(1.0, 4.0)) -> ImagePairWorkload:
    """Plain BAD-256 workload: one 640x480 u8 image, its shifted noisy copy, 1000 keypoints."""
    r_img, r_kp, r_par, r_noise = streams(seed)[:4]
    img1 = quantize_u8(grey_image(r_img, width, height))
    img2 = shifted_noisy_copy(r_noise, img1, 3, 2, 4.0)
    kp1 = keypoints(r_kp, n_kp, width, height, 32.0, scale_range)
    kp2 = shift_keypoints(kp1, 3, 2)
    return ImagePairWorkload("bad256-640x480-1000kp", img1, img2, kp1, kp2,
                             pairs=box_pairs(r_par, n_bits))


def hashsift512_pair(seed: int = SEED_BASE + 1, width: int = 1920, height: int = 1080,
                     n_kp: int = 5000, n_bits: int = 512, scale_range=(1.6, 8.0),
                     with_bad_bits: int = 0) -> ImagePairWorkload:
    """Plain HashSIFT-512 workload: 1920x1080 float32 image in [0, 1], 5000 keypoints.

    With `with_bad_bits` > 0 the workload also carries the u8 rendering of the
    same images and a BAD table, so both descriptors run on one scene."""
    r_img, r_kp, r_par, r_noise, r_bad = streams(seed)[:5]
    grey = grey_image(r_img, width, height)
    img1 = (grey / 255.0).astype(np.float32)
    img2 = shifted_noisy_copy(r_noise, img1, 3, 2, 4.0)
    kp1 = keypoints(r_kp, n_kp, width, height, 32.0, scale_range)
    kp2 = shift_keypoints(kp1, 3, 2)
    B, t = projection(r_par, n_bits)
    w = ImagePairWorkload(f"hashsift{n_bits}-{width}x{height}-{n_kp}kp", img1, img2, kp1, kp2, B=B, t=t)
    if with_bad_bits:
        w.pairs = box_pairs(r_bad, with_bad_bits)
        w.extra["image1_u8"] = quantize_u8(img1.astype(np.float64) * 255.0)
        w.extra["image2_u8"] = quantize_u8(img2.astype(np.float64) * 255.0)
    return w


def batched_sizes(rng: np.random.Generator, n_images: int = 64, w_range=(320, 4000),
                  kp_range=(500, 20000)) -> list[tuple[int, int, int]]:
    """(width, height, n_kp) per image: W ~ U{320..4000}, H = round(0.75 W), n_kp ~ U{500..20000}."""
    out = []
    for _ in range(n_images):
        w = int(rng.integers(w_range[0], w_range[1] + 1))
        h = int(round(0.75 * w))
        out.append((w, h, int(rng.integers(kp_range[0], kp_range[1] + 1))))
    return out


@dataclass
class BatchedWorkload:
    """Scenes of uneven sizes, each with a shifted noisy copy, for batched
    describe-and-match.  images[2i] is scene i and images[2i+1] its copy;
    kps[j] are image j's keypoints (the copy's are the scene's shifted by
    the same (3, 2) px); matches pair each scene with its copy."""

    images: list
    kps: list
    pairs: np.ndarray
    B: np.ndarray
    t: np.ndarray
    matches: list
    sizes: list

    @property
    def total_kp(self) -> int:
        return int(sum(len(k) for k in self.kps))

    def flat_keypoints(self) -> np.ndarray:
        return np.concatenate(self.kps) if self.kps else np.empty(0, dtype=KEYPOINT_DTYPE)


def _batched_scene(seed_seq: np.random.SeedSequence, width: int, height: int, n_kp: int):
    r_img, r_kp, r_noise = [np.random.Generator(np.random.PCG64(s)) for s in seed_seq.spawn(3)]
    img = quantize_u8(grey_image(r_img, width, height))
    copy = shifted_noisy_copy(r_noise, img, 3, 2, 4.0)
    border = min(32.0, 0.25 * min(width, height))
    kp = keypoints(r_kp, n_kp, width, height, border, (1.0, 4.0))
    return img, copy, kp, shift_keypoints(kp, 3, 2)


def batched(seed: int = SEED_BASE + 2, n_images: int = 64, w_range=(320, 4000), kp_range=(500, 20000),
            bad_bits: int = 512, hs_bits: int = 256, sizes=None, workers: int = 8) -> BatchedWorkload:
    """Batched workload: n_images u8 scenes (W ~ U{w_range}, H = 0.75 W; the
    generator of the BAD-256 workload), keypoint counts ~ U{kp_range}, each
    scene with its shifted noisy copy; one BAD table and one HashSIFT
    projection shared by all.  `sizes` overrides the drawn (W, H, n_kp)
    list.  Scenes come from independent seed streams, so generating them
    on `workers` threads gives the same images as generating them in turn."""
    from concurrent.futures import ThreadPoolExecutor

    root = np.random.SeedSequence(seed)
    r_sizes, r_par, r_proj = [np.random.Generator(np.random.PCG64(s)) for s in root.spawn(3)]
    if sizes is None:
        sizes = batched_sizes(r_sizes, n_images, w_range, kp_range)
    scene_seeds = np.random.SeedSequence(seed + 1).spawn(len(sizes))
    with ThreadPoolExecutor(max_workers=max(1, workers)) as pool:
        scenes = list(pool.map(lambda a: _batched_scene(*a),
                               [(scene_seeds[i], w, h, n) for i, (w, h, n) in enumerate(sizes)]))
    images, kps, matches = [], [], []
    for i, (img, copy, kp, kp2) in enumerate(scenes):
        images += [img, copy]
        kps += [kp, kp2]
        matches.append((2 * i, 2 * i + 1))
    B, t = projection(r_proj, hs_bits)
    return BatchedWorkload(images, kps, box_pairs(r_par, bad_bits), B, t, matches, list(sizes))


# --------------------------------------------------------------------------- training triplets


@dataclass
class TripletBatch:
    """n triplets of 32x32 float32 patches (anchor, positive, negative), values in [0, 1]."""

    anchor: np.ndarray
    positive: np.ndarray
    negative: np.ndarray


def _resample_patches(img: np.ndarray, cx, cy, scale, angle) -> np.ndarray:
    """32x32 bilinear crops (scipy.ndimage.map_coordinates, edge-replicated) of img
    around (cx, cy): the patch pixel at row i, column j has the offset
    u = (j - 15.5, i - 15.5) and samples the image at c + scale * Rot(angle) u."""
    from scipy import ndimage

    n = len(cx)
    u = np.arange(32, dtype=np.float64) - 15.5
    uy, ux = np.meshgrid(u, u, indexing="ij")
    c, s = np.cos(angle)[:, None, None], np.sin(angle)[:, None, None]
    sc = scale[:, None, None]
    px = cx[:, None, None] + sc * (c * ux[None] - s * uy[None])
    py = cy[:, None, None] + sc * (s * ux[None] + c * uy[None])
    out = ndimage.map_coordinates(img, [py.reshape(-1), px.reshape(-1)], order=1, mode="nearest")
    return out.reshape(n, 32, 32).astype(np.float32)


def triplets(seed: int = SEED_BASE + 4, n: int = 8192, width: int = 1024, height: int = 768,
             scale_range=(1.0, 4.0), warp_scale=(0.9, 1.1), warp_deg: float = 10.0,
             noise_sigma: float = 0.02) -> TripletBatch:
    """Anchor: crop of a synthetic image at a random keypoint (scale U[1, 4], random
    angle).  Positive: crop of the same source at the keypoint warped by a random
    similarity (scale x U[0.9, 1.1], rotation U[-10, 10] degrees) plus N(0, 0.02^2)
    noise.  Negative: crop at another random keypoint.  Crops are resampled from the
    source image, not from the anchor crop, so warps never extrapolate."""
    r_img, r_kp, r_warp, r_noise, r_neg = streams(seed)[:5]
    img = grey_image(r_img, width, height) / 255.0
    border = 4.0 * 32.0
    cx = r_kp.uniform(border, width - border, n)
    cy = r_kp.uniform(border, height - border, n)
    sc = r_kp.uniform(scale_range[0], scale_range[1], n)
    an = r_kp.uniform(0.0, 2.0 * math.pi, n)
    anchor = _resample_patches(img, cx, cy, sc, an)
    sc2 = sc * r_warp.uniform(warp_scale[0], warp_scale[1], n)
    an2 = an + np.deg2rad(r_warp.uniform(-warp_deg, warp_deg, n))
    positive = _resample_patches(img, cx, cy, sc2, an2)
    positive = np.clip(positive + r_noise.normal(0.0, noise_sigma, positive.shape), 0.0, 1.0).astype(np.float32)
    nx = r_neg.uniform(border, width - border, n)
    ny = r_neg.uniform(border, height - border, n)
    negative = _resample_patches(img, nx, ny, r_neg.uniform(scale_range[0], scale_range[1], n),
                                 r_neg.uniform(0.0, 2.0 * math.pi, n))
    return TripletBatch(anchor, positive, negative)
