"""The C ABI without a GPU: every symbol declared in include/bdesc.h is
exported by libbdesc.so with the binding's signature, and argument
validation (which runs on the host before any HIP call) returns the
documented error codes."""
import ctypes
import os
import re

import pytest

import paper_2108_08380_amd as bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bdesc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bd_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(bd.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return bd.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(L, name), f"{name} declared in bdesc.h but not exported"
    assert set(names) == set(bd.SIGNATURES), "binding signatures out of sync with the header"


def test_header_constants_match_the_binding():
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define (BD_\w+) \(?(-?\d+)\)?", text))
    for name in ("BD_OK", "BD_EINVAL", "BD_EUNSUPPORTED", "BD_ENOMEM", "BD_EDEVICE", "BD_DTYPE_U8", "BD_DTYPE_F32",
                 "BD_PREC_FP32", "BD_PREC_BF16", "BD_PREC_FP8"):
        assert int(defs[name]) == getattr(bd, name), name
    assert int(defs["BD_BATCH_MFMA_MAX_ROWS"]) == bd.MFMA_MAX_ROWS


def test_version_and_error_strings(L):
    assert L.bd_version().decode().startswith("bdesc")
    assert isinstance(L.bd_last_error(), bytes)


def err(L):
    return L.bd_last_error().decode()


def test_context_create_null_output(L):
    assert L.bd_context_create(None, 0) == bd.BD_EINVAL
    assert "null output" in err(L)
    assert L.bd_context_destroy(None) == bd.BD_OK


def test_context_poll_validation(L):
    n = ctypes.c_uint64(5)
    assert L.bd_context_poll(None, None) == bd.BD_EINVAL
    assert "null output" in err(L)
    assert L.bd_context_poll(None, ctypes.byref(n)) == bd.BD_EINVAL
    assert "null context" in err(L) and n.value == 0


def test_build_integral_validation(L):
    p = ctypes.c_void_p(16)  # never dereferenced: validation fails first or the context is null
    assert L.bd_build_integral(None, p, 0, 5, 5, p, 6, None) == bd.BD_EINVAL
    assert "at least 1x1" in err(L)
    assert L.bd_build_integral(None, p, 8, 5, 7, p, 9, None) == bd.BD_EINVAL
    assert "img_pitch" in err(L)
    assert L.bd_build_integral(None, p, 8, 5, 8, p, 8, None) == bd.BD_EINVAL
    assert "ii_pitch" in err(L)
    assert L.bd_build_integral(None, p, 40000, 60000, 40000, p, 40001, None) == bd.BD_EINVAL
    assert "2^31" in err(L)
    assert L.bd_build_integral(None, None, 8, 5, 8, p, 9, None) == bd.BD_EINVAL
    assert "null" in err(L)
    assert L.bd_build_integral(None, p, 8, 5, 8, p, 9, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_build_integral_order_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_build_integral_order(None, p, 0, 5, 5, p, 6, p, 3, p, None) == bd.BD_EINVAL
    assert "at least 1x1" in err(L)
    assert L.bd_build_integral_order(None, p, 8, 5, 7, p, 9, p, 3, p, None) == bd.BD_EINVAL
    assert "img_pitch" in err(L)
    assert L.bd_build_integral_order(None, p, 8, 5, 8, p, 8, p, 3, p, None) == bd.BD_EINVAL
    assert "ii_pitch" in err(L)
    assert L.bd_build_integral_order(None, p, 40000, 60000, 40000, p, 40001, p, 3, p, None) == bd.BD_EINVAL
    assert "2^31" in err(L)
    assert L.bd_build_integral_order(None, p, 8, 5, 8, p, 9, p, -1, p, None) == bd.BD_EINVAL
    assert "n_kp" in err(L)
    assert L.bd_build_integral_order(None, p, 8, 5, 8, p, 9, None, 3, p, None) == bd.BD_EINVAL
    assert "null keypoint" in err(L)
    assert L.bd_build_integral_order(None, p, 8, 5, 8, p, 9, p, 3, None, None) == bd.BD_EINVAL
    assert L.bd_build_integral_order(None, p, 8, 5, 8, p, 9, None, 0, None, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_prepare_view_validation(L):
    p, q = ctypes.c_void_p(16), ctypes.c_void_p(64)

    def call(hs=q, hs_pitch=32, pairs=q, pairs_pitch=64, W=8, H=5, n=3, ctx=None):
        return L.bd_prepare_view(ctx, p, W, H, W, p, W + 1, p, n, p, hs, hs_pitch, pairs, pairs_pitch, None)

    assert call(W=0) == bd.BD_EINVAL and "at least 1x1" in err(L)
    assert call(hs=None) == bd.BD_EINVAL and "together" in err(L)
    assert call(pairs=None) == bd.BD_EINVAL and "together" in err(L)
    assert call(hs_pitch=28) == bd.BD_EINVAL and "hs_pitch" in err(L)
    assert call(hs_pitch=34) == bd.BD_EINVAL and "hs_pitch" in err(L)
    assert call(hs=ctypes.c_void_p(66)) == bd.BD_EINVAL and "hs_pitch" in err(L)
    assert call(pairs_pitch=56) == bd.BD_EINVAL and "pairs_pitch" in err(L)
    assert call(pairs_pitch=68) == bd.BD_EINVAL and "pairs_pitch" in err(L)
    assert call(pairs=ctypes.c_void_p(68)) == bd.BD_EINVAL and "pairs_pitch" in err(L)
    assert call(pairs_pitch=1 << 24) == bd.BD_EINVAL and "2^24" in err(L)
    assert call(n=-1) == bd.BD_EINVAL and "n_kp" in err(L)
    assert call() == bd.BD_EINVAL and "null context" in err(L)
    assert call(hs=None, pairs=None) == bd.BD_EINVAL and "null context" in err(L)


def test_row_pair_image_validation(L):
    p, q = ctypes.c_void_p(16), ctypes.c_void_p(20)
    rp = bd.BD_DTYPE_F32_ROWPAIR
    assert L.bd_hashsift_features(None, p, rp, 10, 10, 72, p, 3, None, p, None) == bd.BD_EINVAL
    assert "row bytes" in err(L)
    assert L.bd_hashsift_features(None, p, rp, 10, 10, 84, p, 3, None, p, None) == bd.BD_EINVAL
    assert "8-byte" in err(L)
    assert L.bd_hashsift_features(None, q, rp, 10, 10, 80, p, 3, None, p, None) == bd.BD_EINVAL
    assert "8-byte" in err(L)
    assert L.bd_hashsift_features(None, p, rp, 10, 10, 80, p, 3, None, p, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_describe_bad_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_describe_bad(None, p, 10, 10, 11, p, 4, None, p, 128, p, None) == bd.BD_EUNSUPPORTED
    assert "n_bits" in err(L)
    assert L.bd_describe_bad(None, p, 10, 10, 10, p, 4, None, p, 256, p, None) == bd.BD_EINVAL
    assert L.bd_describe_bad(None, p, 10, 10, 11, p, -1, None, p, 256, p, None) == bd.BD_EINVAL
    assert L.bd_describe_bad(None, p, 10, 10, 11, None, 4, None, p, 256, p, None) == bd.BD_EINVAL
    # n_kp = 0 needs no pointers, but still a context
    assert L.bd_describe_bad(None, None, 10, 10, 11, None, 0, None, None, 256, None, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_describe_hashsift_validation(L):
    p = ctypes.c_void_p(16)
    base = dict(dtype=bd.BD_DTYPE_F32, W=10, H=10, pitch=40, n=3, n_bits=256, prec=bd.BD_PREC_FP32)

    def call(**kw):
        a = {**base, **kw}
        return L.bd_describe_hashsift(None, p, a["dtype"], a["W"], a["H"], a["pitch"], p, a["n"], None, p, p,
                                      a["n_bits"], a["prec"], a.get("margin", 1e-3), p, None, None, None, None)

    assert call(n_bits=384) == bd.BD_EUNSUPPORTED
    assert call(dtype=7) == bd.BD_EUNSUPPORTED
    assert call(prec=9) == bd.BD_EUNSUPPORTED
    assert call(pitch=39) == bd.BD_EINVAL
    assert call(pitch=42) == bd.BD_EINVAL and "multiple of 4" in err(L)
    assert call(dtype=bd.BD_DTYPE_U8, pitch=10) == bd.BD_EINVAL and "null context" in err(L)
    assert call(n=-2) == bd.BD_EINVAL
    assert call(prec=bd.BD_PREC_BF16, margin=-1.0) == bd.BD_EINVAL and "margin" in err(L)
    assert call(prec=bd.BD_PREC_FP8, margin=float("nan")) == bd.BD_EINVAL
    assert call(prec=bd.BD_PREC_FP8) == bd.BD_EINVAL and "null context" in err(L)


def test_keypoint_order_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_keypoint_order(None, p, 5, 0, 10, p, None) == bd.BD_EINVAL
    assert L.bd_keypoint_order(None, p, -1, 10, 10, p, None) == bd.BD_EINVAL
    assert L.bd_keypoint_order(None, None, 5, 10, 10, p, None) == bd.BD_EINVAL
    assert L.bd_keypoint_order(None, p, 5, 10, 10, p, None) == bd.BD_EINVAL and "null context" in err(L)


def test_hashsift_features_and_project_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_hashsift_features(None, p, 5, 10, 10, 40, p, 3, None, p, None) == bd.BD_EUNSUPPORTED
    assert L.bd_hashsift_features(None, p, bd.BD_DTYPE_F32, 10, 10, 40, None, 3, None, p, None) == bd.BD_EINVAL
    assert L.bd_hashsift_features(None, p, bd.BD_DTYPE_F32, 10, 10, 40, p, 3, None, p, None) == bd.BD_EINVAL
    assert "null context" in err(L)
    assert L.bd_hashsift_project(None, p, None, 3, p, p, 128, bd.BD_PREC_FP32, 0.0, p, None, None, None) == bd.BD_EUNSUPPORTED
    assert L.bd_hashsift_project(None, p, None, 3, p, p, 256, 7, 0.0, p, None, None, None) == bd.BD_EUNSUPPORTED
    assert L.bd_hashsift_project(None, None, None, 3, p, p, 256, bd.BD_PREC_FP32, 0.0, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_hashsift_project(None, p, None, 3, p, p, 256, bd.BD_PREC_FP32, 0.0, p, None, None, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_match_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_match_hamming_knn(None, p, 4, p, 4, 9, 1, p, p, None) == bd.BD_EUNSUPPORTED
    assert L.bd_match_hamming_knn(None, p, 4, p, 4, 4, 3, p, p, None) == bd.BD_EUNSUPPORTED
    assert L.bd_match_hamming_knn(None, p, -1, p, 4, 4, 1, p, p, None) == bd.BD_EINVAL
    assert L.bd_match_hamming_knn(None, p, 4, None, 4, 4, 1, p, p, None) == bd.BD_EINVAL
    assert L.bd_match_hamming_knn(None, p, 4, None, 0, 4, 1, p, p, None) == bd.BD_EINVAL
    assert "null context" in err(L)
    assert L.bd_match_hamming_knn_noalloc(None, p, 4, p, 4, 9, 1, p, p, None) == bd.BD_EUNSUPPORTED
    assert L.bd_match_hamming_knn_noalloc(None, p, 4, p, 4, 4, 3, p, p, None) == bd.BD_EUNSUPPORTED
    assert L.bd_match_hamming_knn_noalloc(None, p, -1, p, 4, 4, 1, p, p, None) == bd.BD_EINVAL
    assert L.bd_match_hamming_knn_noalloc(None, p, 4, None, 4, 4, 1, p, p, None) == bd.BD_EINVAL
    assert L.bd_match_hamming_knn_noalloc(None, p, 4, p, 4, 4, 1, None, p, None) == bd.BD_EINVAL
    assert L.bd_match_hamming_knn_noalloc(None, p, 4, p, 4, 4, 1, p, p, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(bd, "_lib", None)
    monkeypatch.setattr(bd, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        bd.lib()


def test_batch_validation(L):
    p = 16  # never dereferenced: validation fails first or the context is null
    imgs = (bd.BatchImageRec * 2)()
    for i, (W, H, n) in enumerate(((64, 48, 10), (100, 75, 0))):
        imgs[i].img, imgs[i].pitch, imgs[i].W, imgs[i].H, imgs[i].n_kp = p, W, W, H, n
    m = (bd.BatchMatchRec * 1)()
    m[0].query_image, m[0].train_image = 0, 1
    out = ctypes.c_void_p(1)

    def create(images=imgs, n_img=2, matches=m, n_m=1, bad=512, hs=256, prec=bd.BD_PREC_FP32, margin=1e-3, k=2):
        return L.bd_batch_create(None, images, n_img, matches, n_m, bad, hs, prec, margin, k, ctypes.byref(out))

    assert L.bd_batch_create(None, imgs, 2, m, 1, 512, 256, 0, 1e-3, 2, None) == bd.BD_EINVAL
    assert create(n_img=0) == bd.BD_EINVAL and "at least one image" in err(L)
    assert out.value is None  # cleared on error
    assert create(bad=128) == bd.BD_EUNSUPPORTED
    assert create(hs=1024) == bd.BD_EUNSUPPORTED
    assert create(bad=0, hs=0) == bd.BD_EINVAL and "neither" in err(L)
    assert create(prec=5) == bd.BD_EUNSUPPORTED
    assert create(margin=float("inf")) == bd.BD_EINVAL
    assert create(k=3) == bd.BD_EUNSUPPORTED
    m[0].train_image = 2
    assert create() == bd.BD_EINVAL and "names image" in err(L)
    m[0].train_image = 1
    imgs[1].pitch = 99
    assert create() == bd.BD_EINVAL and "pitch" in err(L)
    imgs[1].pitch = 100
    imgs[0].n_kp = -1
    assert create() == bd.BD_EINVAL
    imgs[0].n_kp = 10
    imgs[1].hs_img, imgs[1].hs_dtype, imgs[1].hs_pitch = p, bd.BD_DTYPE_F32, 398
    assert create() == bd.BD_EINVAL and "HashSIFT pitch" in err(L)
    imgs[1].hs_pitch = 400
    imgs[1].hs_dtype = bd.BD_DTYPE_F32_ROWPAIR  # single-image calls only
    assert create() == bd.BD_EUNSUPPORTED and "HashSIFT dtype" in err(L)
    imgs[1].hs_dtype = bd.BD_DTYPE_F32
    imgs[0].W, imgs[0].H, imgs[0].pitch = 50000, 50000, 50000
    assert create() == bd.BD_EINVAL and "32-bit" in err(L)
    imgs[0].W, imgs[0].H, imgs[0].pitch = 64, 48, 64
    assert create() == bd.BD_EINVAL and "null context" in err(L)


def test_batch_tuning_and_run_validation(L):
    tn = bd.BatchTuning()
    assert L.bd_batch_default_tuning(ctypes.byref(tn)) == bd.BD_OK
    assert tn.knn_rows[0] >= 256 and tn.knn_qpl[1] in (0, 1, 2, 4)
    assert L.bd_batch_default_tuning(None) == bd.BD_EINVAL
    assert L.bd_batch_set_tuning(None, ctypes.byref(tn)) == bd.BD_EINVAL
    assert L.bd_batch_get_tuning(None, ctypes.byref(tn)) == bd.BD_EINVAL
    assert L.bd_batch_info(None, None, None) == bd.BD_EINVAL
    assert L.bd_batch_run(None, *([None] * 10), 1, None) == bd.BD_EINVAL
    assert L.bd_batch_autotune(None, *([None] * 10), 3, None) == bd.BD_EINVAL
    assert L.bd_batch_destroy(None) == bd.BD_OK


def test_match_mutual_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_match_mutual(None, p, 4, p, 4, 9, 0.8, p, p, None, None, None) == bd.BD_EUNSUPPORTED
    assert L.bd_match_mutual(None, p, -1, p, 4, 4, 0.8, p, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_match_mutual(None, p, 4, p, 4, 4, -0.5, p, p, None, None, None) == bd.BD_EINVAL
    assert "max_ratio" in err(L)
    assert L.bd_match_mutual(None, p, 4, p, 4, 4, float("nan"), p, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_match_mutual(None, p, 4, p, 4, 4, 0.8, None, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_match_mutual(None, p, 4, None, 4, 4, 0.8, p, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_match_mutual(None, p, 4, None, 0, 4, 0.8, p, p, None, None, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_find_threshold_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_find_threshold(None, p, -1, p, p, 0.5, p, 4, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_find_threshold(None, p, 10, p, p, 0.3, p, 4, p, None, None, None) == bd.BD_EINVAL
    assert "multiple of 1/2" in err(L)
    assert L.bd_find_threshold(None, p, 10, p, p, float("nan"), p, 4, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_find_threshold(None, p, 10, p, p, 0.5, None, 4, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_find_threshold(None, None, 10, p, p, 0.5, p, 4, p, None, None, None) == bd.BD_EINVAL
    assert L.bd_find_threshold(None, p, 10, p, p, 1.5, p, 4, p, None, None, None) == bd.BD_EINVAL
    assert "null context" in err(L)


def test_select_features_validation(L):
    p = ctypes.c_void_p(16)
    call = lambda **kw: L.bd_select_features(None, p, kw.get("P", 100), p, kw.get("N", 50), p, kw.get("J", 10),
                                             kw.get("K", 64), kw.get("tau", 1.0), p, None, None, None, None, None)
    assert call(K=0) == bd.BD_EUNSUPPORTED
    assert call(K=513) == bd.BD_EUNSUPPORTED
    assert call(N=1) == bd.BD_EINVAL
    assert call(N=101) == bd.BD_EINVAL
    assert call(J=0) == bd.BD_EINVAL
    assert call(tau=0.7) == bd.BD_EINVAL
    assert call() == bd.BD_EINVAL and "null context" in err(L)


def test_training_validation(L):
    p = ctypes.c_void_p(16)
    assert L.bd_augment_patches(None, p, 0, p, 4, p, p, p, None) == bd.BD_EINVAL
    assert L.bd_augment_patches(None, p, 10, None, 4, p, p, p, None) == bd.BD_EINVAL
    assert L.bd_augment_patches(None, p, 10, p, 4, p, p, p, None) == bd.BD_EINVAL and "null context" in err(L)

    def step(**kw):
        return L.bd_hashsift_train_step(None, p, kw.get("P", 10), p, kw.get("n", 4), p, p, p, p, kw.get("K", 256), p,
                                        kw.get("step", 1), kw.get("lr", 2e-4), kw.get("tau", 0.5),
                                        kw.get("beta", 1.0), p, None)
    assert step(K=128) == bd.BD_EUNSUPPORTED
    assert step(n=1) == bd.BD_EINVAL
    assert step(step=0) == bd.BD_EINVAL
    assert step(lr=0.0) == bd.BD_EINVAL
    assert step(beta=float("inf")) == bd.BD_EINVAL
    assert step() == bd.BD_EINVAL and "null context" in err(L)


def test_bad_table_validation(L):
    p = ctypes.c_void_p(16)
    out = ctypes.c_void_p(1)
    assert L.bd_bad_table_create(None, p, 256, None, None) == bd.BD_EINVAL
    assert L.bd_bad_table_create(None, p, 128, ctypes.byref(out), None) == bd.BD_EUNSUPPORTED
    assert out.value is None
    assert L.bd_bad_table_create(None, None, 256, ctypes.byref(out), None) == bd.BD_EINVAL
    assert L.bd_bad_table_create(None, p, 256, ctypes.byref(out), None) == bd.BD_EINVAL and "null context" in err(L)
    assert L.bd_bad_table_destroy(None) == bd.BD_OK
    assert L.bd_describe_bad_table(None, p, 10, 10, 11, p, 4, None, None, p, None) == bd.BD_EINVAL
    assert "null table" in err(L)
