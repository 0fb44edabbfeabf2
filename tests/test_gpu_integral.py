"""Integral image on the GPU against the oracle, bit for bit (u32)."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W", [(1, 1), (1, 300), (300, 1), (3, 7), (16, 256), (17, 257), (33, 1000),
                                 (480, 640), (1080, 1920), (241, 4097)])
def test_integral_matches_oracle(ref, dev, H, W):
    rng = np.random.default_rng(H * 7919 + W)
    img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    got = to_np(bd.build_integral(torch.from_numpy(img).to(dev)))
    np.testing.assert_array_equal(got, ref.build_integral(img))


@pytest.mark.parametrize("tail", range(1, 17))
@pytest.mark.parametrize("W", [300, 512])
def test_integral_every_strip_tail(ref, dev, tail, W):
    """The last strip of 16 rows holds 1 .. 16 rows (every tail of a tile),
    on an edge slab (W = 300) and on whole slabs (W = 512)."""
    H = 32 + tail
    img = np.random.default_rng(tail * 31 + W).integers(0, 256, (H, W), dtype=np.uint8)
    got = to_np(bd.build_integral(torch.from_numpy(img).to(dev)))
    np.testing.assert_array_equal(got, ref.build_integral(img))


def test_integral_full_size_batched_image(ref, dev):
    """Largest image of the batched workload: 4000 x 3000 (wraps mod 2^32 nowhere, 3.06e9 < 2^32)."""
    img = np.full((3000, 4000), 255, dtype=np.uint8)
    img[::5, ::3] = np.random.default_rng(5).integers(0, 256, img[::5, ::3].shape, dtype=np.uint8)
    got = to_np(bd.build_integral(torch.from_numpy(img).to(dev)))
    np.testing.assert_array_equal(got, ref.build_integral(img))


def test_integral_wraps_modulo_2_32(ref, dev):
    img = np.full((4300, 4000), 255, dtype=np.uint8)  # total 4.39e9 > 2^32
    got = to_np(bd.build_integral(torch.from_numpy(img).to(dev)))
    exp = ref.build_integral(img)
    np.testing.assert_array_equal(got[-5:], exp[-5:])
    np.testing.assert_array_equal(got[::97], exp[::97])


@pytest.mark.parametrize("pad", [1, 3, 64])
def test_integral_pitched_input_and_output(ref, dev, pad):
    """Row strides that are not multiples of 4 take the byte-load path."""
    rng = np.random.default_rng(pad)
    H, W = 45, 301
    parent = torch.from_numpy(rng.integers(0, 256, (H, W + pad), dtype=np.uint8)).to(dev)
    img = parent[:, :W]
    out_parent = torch.full((H + 1, W + 1 + pad), 7, dtype=torch.uint32, device=dev)
    out = out_parent[:, : W + 1]
    bd.build_integral(img, out=out)
    got = to_np(out_parent)
    np.testing.assert_array_equal(got[:, : W + 1], ref.build_integral(to_np(img)))
    assert (got[:, W + 1:] == 7).all(), "wrote outside the output rows"


def test_integral_config_workload(ref, dev):
    w = synth.bad256_pair()
    for img in (w.image1, w.image2):
        got = to_np(bd.build_integral(torch.from_numpy(img).to(dev)))
        np.testing.assert_array_equal(got, ref.build_integral(img))


def test_integral_deterministic(dev):
    img = torch.randint(0, 256, (777, 1333), dtype=torch.uint8, device=dev)
    a = to_np(bd.build_integral(img))
    b = to_np(bd.build_integral(img))
    np.testing.assert_array_equal(a, b)


def test_integral_near_the_index_limit(ref, dev):
    """32767 x 32768 (1.07e9 integral elements, the largest power-of-two width
    under the 2^31-element limit of bd_build_integral): sampled rows and the
    last row against the oracle, total sum modulo 2^32."""
    H, W = 32767, 32768
    rng = np.random.default_rng(77)
    img = np.full((H, W), 200, dtype=np.uint8)
    img[rng.integers(0, H, 4096), :] = rng.integers(0, 256, (4096, W), dtype=np.uint8)
    d_img = torch.from_numpy(img).to(dev)
    ii = bd.build_integral(d_img)
    del d_img
    exp = ref.build_integral(img)
    iv = ii.view(torch.int32)  # torch indexes no uint32 device tensors; same bits
    rows = [0, 1, 17, 4096, H // 2, H - 1, H]
    got_rows = iv[rows].cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got_rows, exp[rows])
    cols = torch.from_numpy(rng.integers(0, W + 1, 64)).to(dev)
    np.testing.assert_array_equal(iv[:, cols].cpu().numpy().view(np.uint32), exp[:, cols.cpu().numpy()])
    assert int(got_rows[-1, -1]) == int(img.sum(dtype=np.uint64) % (1 << 32))


@pytest.mark.parametrize("W", [255, 256, 257, 512, 700, 1023, 1024])
@pytest.mark.parametrize("aligned_rows", [True, False])
def test_integral_row_alignment(ref, dev, W, aligned_rows):
    """16-byte aligned output rows (row stride a multiple of 4) take the
    full-width store path, with the boundary column shared by neighbouring
    tiles and column W written by the rightmost tile; other strides store
    per column.  Both equal the oracle and leave the row padding untouched."""
    H = 37
    rng = np.random.default_rng(W * 3 + aligned_rows)
    img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    pitch = (W + 1 + 3) // 4 * 4 + 4 if aligned_rows else (W + 1) | 1
    if not aligned_rows and pitch % 4 == 0:
        pitch += 1
    parent = torch.full((H + 1, pitch), 7, dtype=torch.uint32, device=dev)
    out = parent[:, : W + 1]
    bd.build_integral(torch.from_numpy(img).to(dev), out=out)
    got = to_np(parent)
    np.testing.assert_array_equal(got[:, : W + 1], ref.build_integral(img))
    assert (got[:, W + 1:] == 7).all(), "wrote outside the output rows"


def test_integral_default_buffer_is_aligned(dev):
    ii = bd.build_integral(torch.zeros((5, 300), dtype=torch.uint8, device=dev))
    assert ii.shape == (6, 301) and ii.stride(0) % 4 == 0 and ii.data_ptr() % 16 == 0
