"""Describe-and-match throughput on one MI355X.

One step is the whole hot path over one image pair of 1920x1080 pixels
with 5000 keypoints per view (keypoint scale U[1.6, 8], random angle):
  spatial processing order of both keypoint sets,
  integral image of both u8 views, BAD-256 codes for both views,
  HashSIFT-512 codes for both float32 views (features + FP32-MFMA
  projection), Hamming 2-NN of view 1 against view 2 for both code types.
Inputs are seeded synthetic images shaped like the paper's timing workload
and are resident in HBM before timing starts.  `value` counts keypoints
described (both descriptors) and matched per second.

The JSON line also carries per-stage HIP-event timings, the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample of the same
workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 64 lanes x 2.4 GHz: one 32-bit VALU op per lane per clock (not packed)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
FP32_MFMA_PEAK_TFLOPS = 157.3
INT8_MFMA_PEAK_TOPS = 5000.0  # dense int8 MFMA, 5.0 POP/s

W, H, N_KP = 1920, 1080, 5000
BAD_BITS, HS_BITS, K = 256, 512, 2


def parse():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--graph", type=int, default=1, help="replay the step as a captured HIP graph (1) or eager (0)")
    p.add_argument("--stage-reps", type=int, default=50)
    p.add_argument("--cpu-sample", type=int, default=2500, help="keypoints per view for the CPU oracle sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-batched", action="store_true", help="skip the 128-image batched workload")
    p.add_argument("--batched-only", action="store_true", help="run only the batched workload and print its JSON")
    p.add_argument("--precision-only", action="store_true",
                   help="run only the 200000-row FP32/BF16/FP8 projection comparison and print its JSON")
    p.add_argument("--step-only", action="store_true", help="only the step, its stage timings and the checks")
    p.add_argument("--only", default="", help="profile helper: run only this stage in the step loop")
    p.add_argument("--copy-calibration-mb", type=int, default=0,
                   help="run a plain device copy of this many MiB five times and exit (HBM counter calibration)")
    return p.parse_args()


class Workload:
    def __init__(self, dev):
        import torch

        import paper_2108_08380_amd as bd
        from paper_2108_08380_amd import synth

        w = synth.hashsift512_pair(synth.SEED_BASE + 1, W, H, N_KP, HS_BITS, with_bad_bits=BAD_BITS)
        self.host = w
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.u8 = [T(w.extra["image1_u8"]), T(w.extra["image2_u8"])]
        self.f32 = [T(w.image1), T(w.image2)]
        self.kps = [bd.keypoints_tensor(w.kp1, dev), bd.keypoints_tensor(w.kp2, dev)]
        self.pairs = bd.pairs_tensor(w.pairs, dev)
        self.table = bd.BadTable(self.pairs)  # compiled once, like a plan
        self.B, self.t = T(w.B), T(w.t)
        self.order = [torch.empty((N_KP,), dtype=torch.int32, device=dev) for _ in range(2)]
        self.ii = [bd.integral_buffer(H, W, dev) for _ in range(2)]
        # row-pair copies of the HashSIFT images, written by prepare_view in every step
        self.rp = [torch.empty((H, W, 2), dtype=torch.float32, device=dev) for _ in range(2)]
        self.bad = [torch.empty((N_KP, BAD_BITS // 64), dtype=torch.uint64, device=dev) for _ in range(2)]
        self.hist = [torch.empty((N_KP, 128), dtype=torch.float32, device=dev) for _ in range(2)]
        self.hs = [torch.empty((N_KP, HS_BITS // 64), dtype=torch.uint64, device=dev) for _ in range(2)]
        self.idx = [torch.empty((N_KP, K), dtype=torch.int32, device=dev) for _ in range(2)]
        self.dist = [torch.empty((N_KP, K), dtype=torch.uint32, device=dev) for _ in range(2)]

    # the stages of one step, each a list of library calls
    def stages(self):
        import paper_2108_08380_amd as bd

        s = self
        return {
            "keypoint_order": lambda: [bd.keypoint_order(s.kps[v], W, H, out=s.order[v]) for v in (0, 1)],
            "integral": lambda: [bd.build_integral(s.u8[v], out=s.ii[v]) for v in (0, 1)],
            "bad_describe": lambda: [bd.describe_bad(s.ii[v], s.kps[v], out=s.bad[v], order=s.order[v], table=s.table)
                                     for v in (0, 1)],
            "hashsift_features": lambda: [bd.hashsift_features(s.rp[v], s.kps[v], out=s.hist[v], order=s.order[v])
                                          for v in (0, 1)],
            "hashsift_project": lambda: [bd.hashsift_project(s.hist[v], s.B, s.t, s.kps[v], out=s.hs[v]) for v in (0, 1)],
            "match_bad256": lambda: bd.match_hamming_knn(s.bad[0], s.bad[1], K, s.idx[0], s.dist[0]),
            "match_hashsift512": lambda: bd.match_hamming_knn(s.hs[0], s.hs[1], K, s.idx[1], s.dist[1]),
        }

    def describe(self, v):
        import paper_2108_08380_amd as bd

        s = self
        bd.prepare_view(s.u8[v], s.kps[v], s.f32[v], out=s.ii[v], order=s.order[v], pairs=s.rp[v])
        bd.describe_bad(s.ii[v], s.kps[v], out=s.bad[v], order=s.order[v], table=s.table)
        bd.hashsift_features(s.rp[v], s.kps[v], out=s.hist[v], order=s.order[v])
        bd.hashsift_project(s.hist[v], s.B, s.t, s.kps[v], out=s.hs[v])

    def step(self, only=""):
        """One step.  The two views are described on two streams (view 1 on a
        side stream forked from the current one), then the two code types
        are matched on the two streams; each stream has its own library
        context.  Inside graph capture the fork becomes two graph branches."""
        import torch

        import paper_2108_08380_amd as bd

        if only:
            for name, fn in self.stages().items():
                if name == only:
                    fn()
            return
        cur = torch.cuda.current_stream()
        if not hasattr(self, "side"):
            self.side = torch.cuda.Stream()
        self.side.wait_stream(cur)
        with torch.cuda.stream(self.side):
            self.describe(1)
        self.describe(0)
        cur.wait_stream(self.side)
        self.side.wait_stream(cur)
        with torch.cuda.stream(self.side):
            bd.match_hamming_knn(self.hs[0], self.hs[1], K, self.idx[1], self.dist[1])
        bd.match_hamming_knn(self.bad[0], self.bad[1], K, self.idx[0], self.dist[0])
        cur.wait_stream(self.side)


# algorithmic work per launch of each stage's main kernel: what the stage's
# definition requires per keypoint, pixel or pair, not what the kernel executes
def stage_work():
    px = W * H
    return {
        # keypoint order: 16 bytes read + 4 bytes written per keypoint
        "keypoint_order": ("hbm", 20.0 * N_KP, "GB/s"),
        # integral image: 1 byte read + 4 bytes written per pixel, per view
        "integral": ("hbm", 5.0 * px, "GB/s"),
        # BAD: HBM-unique bytes are keypoints + codes + the integral image once
        "bad_describe": ("hbm", 16.0 * N_KP + BAD_BITS / 8 * N_KP + 4.0 * (px + W + H + 1), "GB/s"),
        # HashSIFT features: ~67k ALU ops per keypoint (1156 bilinear samples x 14, 1024 pixels x 50)
        "hashsift_features": ("alu", (1156 * 14 + 1024 * 50) * N_KP, "TOP/s"),
        # projection: 2 * n_bits * 128 flops per keypoint on FP32 MFMA
        "hashsift_project": ("mfma", 2.0 * HS_BITS * 128 * N_KP, "TFLOP/s"),
        # Hamming on int8 MFMA: per pair one multiply-add per code bit (2 ops)
        "match_bad256": ("mfma", 2.0 * BAD_BITS * float(N_KP) * N_KP, "TOP/s", INT8_MFMA_PEAK_TOPS),
        "match_hashsift512": ("mfma", 2.0 * HS_BITS * float(N_KP) * N_KP, "TOP/s", INT8_MFMA_PEAK_TOPS),
    }


# HBM bytes per launch of each stage (sum over its kernels), from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
#   bench.py --step-only --steps 2 --warmup 1 --stage-reps 2 --graph 0
# scaled by the same counters on a plain 256 MiB device copy (FETCH_SIZE
# reads half the copied bytes: x2 KiB -> 2048 bytes; WRITE_SIZE exact:
# 1024 bytes per KiB).  A value is reported only while the stage's source
# files still have the recorded SHA-256 prefix (of their concatenation): any
# change to the kernels invalidates the counters.
PMC_TRAFFIC = {
    "keypoint_order": (("order.hip", "order_body.hpp"), "b6dbfa27dc112f78", 44 * 2048 + 20 * 1024),
    "integral": ("integral.hip", "db3e519d3c76c709", (1072 + 1806) * 2048 + (971 + 8159) * 1024),
    "bad_describe": ("bad.hip", "73b96b61b0287a2a", 9644 * 2048 + 161 * 1024),
    "hashsift_features": ("hashsift.hip", "73d50dc3bf827b93", 16993 * 2048 + 2500 * 1024),
    "hashsift_project": ("hashsift.hip", "73d50dc3bf827b93", 2367 * 2048 + 312 * 1024),
    "match_bad256": ("hamming.hip", "b45b06214a9c6ad9", (882 + 300) * 2048 + (469 + 78) * 1024),
    "match_hashsift512": ("hamming.hip", "b45b06214a9c6ad9", (1684 + 300) * 2048 + (469 + 78) * 1024),
}


# Vector-L1 (TCP) cache accesses per launch, from rocprofv3 --pmc
# TCP_TOTAL_CACHE_ACCESSES_sum on the same launch (a gather instruction counts
# one access per lane).  The L1 of a CU serves about one scattered lane access
# per clock (lanes of one instruction that fall in the same cache line can be
# served together, so a gather with some locality can pass 1 slightly), so
# accesses / (duration x 256 CUs x 2.4 GHz) is the kernel's fraction of that
# rate.
PMC_L1_ACCESSES = {
    "hashsift_features": ("hashsift.hip", "73d50dc3bf827b93", 5975756),
    "bad_describe": ("bad.hip", "73b96b61b0287a2a", 10315006),
}
L1_ACCESS_PEAK_PER_S = 256 * 2.4e9


def pmc_traffic(stage, table=None):
    """Measured HBM bytes (or another counter of `table`) per launch of a
    stage, or None once its source changed."""
    import hashlib

    entry = (PMC_TRAFFIC if table is None else table).get(stage)
    if entry is None:
        return None
    fnames, digest, nbytes = entry
    if isinstance(fnames, str):
        fnames = (fnames,)
    try:
        data = b"".join(open(os.path.join(ROOT, "paper_2108_08380_amd", "csrc", f), "rb").read() for f in fnames)
    except OSError:
        return None
    cur = hashlib.sha256(data).hexdigest()[:16]
    return nbytes if cur == digest else None


def peak_of(bound):
    """Default peak of a bound: HBM bandwidth, VALU lane-ops, FP32 MFMA (a
    stage of another MFMA type names its own peak in stage_work)."""
    return {"hbm": HBM_PEAK_GBS, "alu": ALU_PEAK_TOPS, "mfma": FP32_MFMA_PEAK_TFLOPS}[bound]


PER_VIEW_STAGES = ("keypoint_order", "integral", "bad_describe", "hashsift_features", "hashsift_project")


def time_stages(wl, reps):
    """Per-launch duration of each stage, with HIP events on the launch stream:
    (average over `reps` back-to-back repetitions, median and minimum of
    `reps` repetitions timed one by one)."""
    import torch

    out = {}
    stream = torch.cuda.current_stream()
    for name, fn in wl.stages().items():
        fn()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(reps):
            fn()
        end.record(stream)
        end.synchronize()
        # two launches per rep for per-view stages
        launches = 2 if name in PER_VIEW_STAGES else 1
        avg = start.elapsed_time(end) / reps / launches
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for r in range(reps):
            fn()
            ev[r + 1].record(stream)
        ev[-1].synchronize()
        each = sorted(ev[r].elapsed_time(ev[r + 1]) / launches for r in range(reps))
        out[name] = (avg, float(np.median(each)), each[0])
    return out


def roof_ms(bound, units, peak):
    """Time of `units` of work at `peak` (GB/s for hbm, T ops/s otherwise), in ms."""
    return units / (peak * (1e9 if bound == "hbm" else 1e12)) * 1e3


def graph_time(fn, reps=100, warmup=5):
    """ms per replay of `fn` captured as one HIP graph (after eager warm-up)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        fn()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        fn()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        g.replay()
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / reps


def describe_rates(wl, reps=200):
    """Keypoints described per second on the step's workload without matching:
    describe-only (keypoint order, BAD from the integral images, HashSIFT),
    integral + describe, and each descriptor alone, both views on two streams
    as in the step, each timed as a graph replay."""
    import torch

    def two_views(body):
        def run():
            cur = torch.cuda.current_stream()
            if not hasattr(wl, "side_d"):
                wl.side_d = torch.cuda.Stream()
            wl.side_d.wait_stream(cur)
            with torch.cuda.stream(wl.side_d):
                body(1)
            body(0)
            cur.wait_stream(wl.side_d)
        return run

    import paper_2108_08380_amd as bd

    def order(v):
        bd.keypoint_order(wl.kps[v], W, H, out=wl.order[v])

    def integral_order(v):
        bd.build_integral_order(wl.u8[v], wl.kps[v], out=wl.ii[v], order=wl.order[v])

    def bad(v):
        bd.describe_bad(wl.ii[v], wl.kps[v], out=wl.bad[v], order=wl.order[v], table=wl.table)

    def prepare(v):
        bd.prepare_view(wl.u8[v], wl.kps[v], wl.f32[v], out=wl.ii[v], order=wl.order[v], pairs=wl.rp[v])

    def hs(v, img=None):
        img = wl.f32[v] if img is None else img
        bd.hashsift_features(img, wl.kps[v], out=wl.hist[v], order=wl.order[v])
        bd.hashsift_project(wl.hist[v], wl.B, wl.t, wl.kps[v], out=wl.hs[v])

    variants = {
        "describe_only": lambda v: (order(v), bad(v), hs(v)),
        "integral_plus_describe": lambda v: (prepare(v), bad(v), hs(v, wl.rp[v])),
        "bad256_only": lambda v: (order(v), bad(v)),
        "integral_plus_bad256": lambda v: (integral_order(v), bad(v)),
        "hashsift512_only": lambda v: (order(v), hs(v)),
    }
    out = {}
    for name, body in variants.items():
        ms = graph_time(two_views(body), reps)
        out[name] = {"ms": round(ms, 4), "keypoints_per_s": round(2 * N_KP / (ms * 1e-3), 1)}
    return out


def config0_step(dev, reps=200):
    """The plain BAD-256 workload: one 640x480 u8 image pair, 1000 keypoints per
    view (scale U[1, 4]), 256 box pairs; integral images and BAD-256 of both
    views, then Hamming 1-NN 1000x1000, as one graph replay (the two views on
    two streams).  Also the describe-only and integral + describe parts."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import synth

    w = synth.bad256_pair(synth.SEED_BASE + 0)
    Hc, Wc = w.image1.shape
    n = len(w.kp1)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    imgs = [T(w.image1), T(w.image2)]
    kps = [bd.keypoints_tensor(w.kp1, dev), bd.keypoints_tensor(w.kp2, dev)]
    pairs = bd.pairs_tensor(w.pairs, dev)
    table = bd.BadTable(pairs)
    order = [torch.empty((n,), dtype=torch.int32, device=dev) for _ in range(2)]
    ii = [bd.integral_buffer(Hc, Wc, dev) for _ in range(2)]
    codes = [torch.empty((n, 4), dtype=torch.uint64, device=dev) for _ in range(2)]
    idx = torch.empty((n, 1), dtype=torch.int32, device=dev)
    dist = torch.empty((n, 1), dtype=torch.uint32, device=dev)
    side = torch.cuda.Stream()

    def view(v, integral=True):
        if integral:
            bd.build_integral_order(imgs[v], kps[v], out=ii[v], order=order[v])
        else:
            bd.keypoint_order(kps[v], Wc, Hc, out=order[v])
        bd.describe_bad(ii[v], kps[v], out=codes[v], order=order[v], table=table)

    def run(integral=True, match=True):
        cur = torch.cuda.current_stream()
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            view(1, integral)
        view(0, integral)
        cur.wait_stream(side)
        if match:
            bd.match_hamming_knn(codes[0], codes[1], 1, idx, dist)

    ms = graph_time(run, reps)
    ms_desc = graph_time(lambda: run(False, False), reps)
    ms_int_desc = graph_time(lambda: run(True, False), reps)
    torch.cuda.synchronize()
    true_rate = float((idx[:, 0] == torch.arange(n, device=dev, dtype=torch.int32)).float().mean())
    return {
        "workload": f"BAD-256, {Wc}x{Hc} u8 image pair, {n} keypoints per view, Hamming 1-NN {n}x{n}",
        "ms_per_step": round(ms, 4),
        "keypoints_per_s": round(2 * n / (ms * 1e-3), 1),
        "hamming_pairs_per_s": round(n * n / (ms * 1e-3), 1),
        "describe_only": {"ms": round(ms_desc, 4), "keypoints_per_s": round(2 * n / (ms_desc * 1e-3), 1)},
        "integral_plus_describe": {"ms": round(ms_int_desc, 4),
                                   "keypoints_per_s": round(2 * n / (ms_int_desc * 1e-3), 1)},
        "true_match_rate": round(true_rate, 4),
    }


def hbm_copy_rate(dev, mib=1024, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes per second)
    of a `mib` MiB buffer, the denominator the HBM fractions can be read
    against beside the 8 TB/s specification."""
    import torch

    n = mib << 20
    src = torch.empty((n,), dtype=torch.uint8, device=dev)
    src.fill_(7)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(src)
    end.record()
    end.synchronize()
    ms = start.elapsed_time(end) / reps
    del src, dst
    return {"bytes_per_copy": 2 * n, "ms": round(ms, 4), "gbs": round(2 * n / (ms * 1e-3) / 1e9, 1),
            "spec_gbs": HBM_PEAK_GBS}


def precision_projection(wl, n_rows=200000, reps=20):
    """HashSIFT-512 projection of 200000 feature rows (the bench features tiled)
    in FP32, BF16 and FP8 with the 1e-3 FP32 re-check margin: time per launch,
    flipped bits and largest response change against the FP32 path."""
    import torch

    import paper_2108_08380_amd as bd

    f = torch.cat(wl.hist, 0)
    f = f.repeat((n_rows + f.shape[0] - 1) // f.shape[0], 1)[:n_rows].contiguous()
    out = {}
    ref_codes = ref_resp = None
    for prec in ("fp32", "bf16", "fp8"):
        cnt = torch.zeros(1, dtype=torch.uint32, device=f.device)
        codes, resp = bd.hashsift_project(f, wl.B, wl.t, precision=prec, with_resp=True, recheck_count=cnt)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            bd.hashsift_project(f, wl.B, wl.t, precision=prec, out=codes)
        e.record()
        e.synchronize()
        ms = s.elapsed_time(e) / reps
        flops = 2.0 * HS_BITS * 128 * n_rows
        item = {"ms_per_launch": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2)}
        if ref_codes is None:
            ref_codes, ref_resp = codes, resp
        else:
            x = (codes.view(torch.int64) ^ ref_codes.view(torch.int64)).cpu().numpy()
            flips = int(np.unpackbits(x.view(np.uint8)).sum())
            item["flipped_bits_vs_fp32"] = flips
            item["flip_rate_vs_fp32"] = flips / (n_rows * HS_BITS)
            item["rechecked_responses"] = int(cnt.cpu()[0])
            item["max_abs_response_change_vs_fp32"] = float((resp - ref_resp).abs().max())
        out[prec] = item
    return out


def differentiation_step(dev, n=8192, reps=5):
    """One training step of the differentiation extension on 8192 triplets of
    32x32 patches: relaxed BAD-512 and HashSIFT-512 descriptors of anchors and
    positives, hardest-negative triplet loss (8192 x 8192 similarities), and
    the full backward pass to the parameters.  Times per step (HIP events)."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import autograd as ag
    from paper_2108_08380_amd import synth

    b = synth.triplets(synth.SEED_BASE + 4, n=n)
    rng = np.random.default_rng(0)
    pairs = bd.pairs_tensor(synth.box_pairs(rng, 512), dev)
    an = torch.from_numpy(b.anchor).to(dev)
    po = torch.from_numpy(b.positive).to(dev)
    w1 = torch.ones(512, device=dev, requires_grad=True)
    w2 = torch.ones(512, device=dev, requires_grad=True)
    th = torch.zeros(512, device=dev, requires_grad=True)
    Bm, tv = synth.projection(rng, 512)
    B = torch.from_numpy(Bm).to(dev).requires_grad_()
    t = torch.from_numpy(tv).to(dev).requires_grad_()
    fa, fp = bd.hashsift_patch_features(an), bd.hashsift_patch_features(po)

    def bad_step():
        loss = ag.bad_triplet_loss(an, po, w1, w2, th, pairs)
        loss.backward()
        return loss

    def hs_step():
        loss = ag.hashsift_triplet_loss(fa, fp, B, t)
        loss.backward()
        return loss

    out = {}
    for name, fn in (("bad512", bad_step), ("hashsift512", hs_step)):
        loss = fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        out[name] = {"ms_per_step": round(s.elapsed_time(e) / reps, 3), "loss": round(float(loss.detach()), 6)}
    # the similarity tiles alone: 2 * n^2 * K flops on FP32 MFMA
    D_a = torch.tanh(torch.randn(n, 512, device=dev))
    D_p = torch.tanh(torch.randn(n, 512, device=dev))
    bd.trl_hnm_fwd(D_a, D_p, 0.5)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        bd.trl_hnm_fwd(D_a, D_p, 0.5)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    out["trl_forward_ms"] = round(ms, 3)
    out["trl_forward_tflops"] = round(2.0 * n * n * 512 / (ms * 1e-3) / 1e12, 2)
    return out


def pair_via_batch(wl, reps=200):
    """The same step (both views, both descriptors, both matchers) through the
    batched entry point: one launch per stage for the two views, captured as
    one graph.  Outputs are compared with the single-image step's."""
    import torch

    import paper_2108_08380_amd as bd

    kps = torch.cat(wl.kps).contiguous()
    b = bd.Batch(wl.u8, [N_KP, N_KP], [(0, 1)], bad_bits=BAD_BITS, hs_bits=HS_BITS, k=K, hs_images=wl.f32)
    out = b.allocate_outputs()
    tuning = b.autotune(kps, wl.pairs, wl.B, wl.t, out=out, reps=5)
    b.run(kps, wl.pairs, wl.B, wl.t, out=out, graph=True)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.run(kps, wl.pairs, wl.B, wl.t, out=out, graph=True)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    same = (torch.equal(out["bad_codes"], torch.cat(wl.bad)) and torch.equal(out["hs_codes"], torch.cat(wl.hs))
            and torch.equal(out["bad_idx"], wl.idx[0]) and torch.equal(out["bad_dist"], wl.dist[0])
            and torch.equal(out["hs_idx"], wl.idx[1]) and torch.equal(out["hs_dist"], wl.dist[1]))
    b.close()
    return {"ms_per_step": round(ms, 4), "keypoints_per_s": round(2 * N_KP / (ms * 1e-3), 1),
            "bit_identical_to_single_image_step": bool(same), "tuning": tuning}


def mutual_matching(wl, reps=20):
    """Mutual nearest neighbours + ratio 0.8 (two k-NN passes and the cross
    check) on the step's BAD-256 and HashSIFT-512 codes of the two views:
    time per call, matches kept and their true-correspondence rate."""
    import torch

    import paper_2108_08380_amd as bd

    out = {}
    ar = torch.arange(N_KP, device=wl.bad[0].device, dtype=torch.int32)
    for name, codes in (("bad256", wl.bad), ("hashsift512", wl.hs)):
        match, dist, count = bd.match_mutual(codes[0], codes[1], 0.8, with_count=True)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            bd.match_mutual(codes[0], codes[1], 0.8)
        e.record()
        e.synchronize()
        kept = match >= 0
        out[name] = {"ms_per_call": round(s.elapsed_time(e) / reps, 4), "matches": int(count.cpu()[0]),
                     "true_rate": round(float((match[kept] == ar[kept]).float().mean()), 4)}
    return out


def threshold_search(dev, n=16384, J=1000, reps=5):
    """Alg. 2 (threshold search) for J = 1000 candidate BAD features, the
    paper's per-round candidate count, over n triplets of u8 32x32 patches:
    time per call and candidate-patch features per second."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import synth

    b = synth.triplets(synth.SEED_BASE + 4, n=n)
    p = np.empty((3 * n, 32, 32), dtype=np.float32)
    p[0::3], p[1::3], p[2::3] = b.anchor, b.positive, b.negative
    patches = torch.from_numpy(np.clip(np.rint(p * 255.0), 0, 255).astype(np.uint8)).to(dev)
    rng = np.random.default_rng(7)
    s_ap = torch.from_numpy(rng.integers(-64, 65, n).astype(np.int32)).to(dev)
    s_an = torch.from_numpy(rng.integers(-64, 65, n).astype(np.int32)).to(dev)
    cands = bd.pairs_tensor(synth.box_pairs(rng, J, radius_range=(0, 7)), dev)
    bd.find_threshold(patches, s_ap, s_an, 1.0, cands)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        bd.find_threshold(patches, s_ap, s_an, 1.0, cands)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    return {"triplets": n, "candidates": J, "bins": 5110, "ms_per_call": round(ms, 3),
            "candidate_patch_features_per_s": round(3.0 * n * J / (ms * 1e-3), 1)}


def greedy_selection(dev, P=16384, N=8192, J=1000, K=256):
    """Alg. 1: learning a BAD-256 table by greedy selection on a pool of P
    matched u8 patch pairs, each of the K = 256 rounds with N sampled pairs
    (in-batch hardest negatives with anchor swap on the bits so far) and
    J = 1000 random candidate box pairs (the paper's J).  One run, timed with
    HIP events; loss of the first and last rounds."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import synth

    b = synth.triplets(synth.SEED_BASE + 5, n=P)
    pool = np.empty((2 * P, 32, 32), dtype=np.uint8)
    pool[0::2] = np.clip(np.rint(b.anchor * 255), 0, 255)
    pool[1::2] = np.clip(np.rint(b.positive * 255), 0, 255)
    rng = np.random.default_rng(11)
    samples = np.stack([rng.permutation(P)[:N] for _ in range(K)]).astype(np.int32)
    cands = synth.box_pairs(rng, K * J, radius_range=(0, 7)).view(np.uint8).reshape(K, J, 12)
    pool_t = torch.from_numpy(pool).to(dev)
    samples_t = torch.from_numpy(samples).to(dev)
    cands_t = torch.from_numpy(cands).to(dev)
    bd.select_features(pool_t, samples_t[:2].contiguous(), cands_t[:2].contiguous())  # warm-up, workspace
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    table, chosen, cbin, loss, codes = bd.select_features(pool_t, samples_t, cands_t)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e)
    loss = loss.cpu().numpy()
    return {"pool_pairs": P, "sampled_pairs_per_round": N, "candidates_per_round": J, "rounds": K,
            "ms_total": round(ms, 2), "ms_per_round": round(ms / K, 3),
            "loss_first_round": float(loss[0]), "loss_last_round": float(loss[-1])}


def hashsift_training(dev, P=16384, n=8192, K=512, iters=50):
    """HashSIFT training (Sec. III-B): Adam (lr 2e-4) on a 512 x 128 projection
    from N(0, 0.25), batches of 8192 augmented pairs (the differentiation
    workload's batch size) with in-batch hardest negatives; time per
    iteration (augment, features, relaxed descriptors, loss, backward,
    update) and the loss trend."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import synth

    b = synth.triplets(synth.SEED_BASE + 6, n=P)
    pool = np.empty((2 * P, 32, 32), np.float32)
    pool[0::2], pool[1::2] = b.anchor, b.positive
    pool = torch.from_numpy(pool).to(dev)
    rng = np.random.default_rng(12)
    batches, params, noise = [], [], []
    for _ in range(4):  # a few pre-drawn batches, reused in turn
        batches.append(torch.from_numpy(rng.permutation(P)[:n].astype(np.int32)).to(dev))
        params.append(torch.from_numpy(np.stack([rng.uniform(-0.17, 0.17, 2 * n), rng.uniform(0.9, 1.1, 2 * n),
                                                 rng.uniform(0.8, 1.2, 2 * n), rng.uniform(-0.1, 0.1, 2 * n),
                                                 rng.uniform(0.0, 1.0, 2 * n)], axis=1).astype(np.float32)).to(dev))
        noise.append(torch.from_numpy(rng.normal(0, 0.02, (2 * n, 32, 32)).astype(np.float32)).to(dev))
    tr = bd.HashSIFTTrainer(K, dev, seed=1)
    first = float(tr.train_step(pool, batches[0], params[0], noise[0]).cpu()[0])
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for it in range(iters):
        j = it % 4
        loss = tr.train_step(pool, batches[j], params[j], noise[j])
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / iters
    return {"batch_pairs": n, "n_bits": K, "iterations": iters + 1, "ms_per_iteration": round(ms, 3),
            "pairs_per_s": round(n / (ms * 1e-3), 1), "loss_first": round(first, 5),
            "loss_last": round(float(loss.cpu()[0]), 5)}


def batched_step(dev, reps=5):
    """The batching extension on its full workload: 64 u8 scenes of
    320x240 .. 4000x3000 pixels with 500 .. 20000 keypoints, each with its
    shifted noisy copy (128 images), BAD-512 + HashSIFT-256 and per-scene
    Hamming 2-NN against the copy for both code types.  The batch is
    autotuned, then replayed as one captured graph (HIP events around
    `reps` replays) and compared, output for output, with the single-image
    entry points run image by image on the same GPU (timed the same way)."""
    import torch

    import paper_2108_08380_amd as bd
    from paper_2108_08380_amd import synth

    w = synth.batched(workers=16)
    imgs = [torch.from_numpy(im).to(dev) for im in w.images]
    kps = bd.keypoints_tensor(w.flat_keypoints(), dev)
    pairs = bd.pairs_tensor(w.pairs, dev)
    B, t = torch.from_numpy(w.B).to(dev), torch.from_numpy(w.t).to(dev)
    n_kp = [len(k) for k in w.kps]
    b = bd.Batch(imgs, n_kp, w.matches, bad_bits=512, hs_bits=256, k=2)
    out = b.allocate_outputs()
    t0 = time.perf_counter()
    tuning = b.autotune(kps, pairs, B, t, out=out, reps=2)
    tune_s = time.perf_counter() - t0

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        return s.elapsed_time(e) / reps

    ms_batch = timed(lambda: b.run(kps, pairs, B, t, out=out, graph=True))

    offs = np.concatenate([[0], np.cumsum(n_kp)])
    kp_views = [kps[offs[j]:offs[j + 1]] for j in range(len(imgs))]
    iis = [bd.integral_buffer(im.shape[0], im.shape[1], dev) for im in imgs]
    plain = {"bad": [torch.empty((n, 8), dtype=torch.uint64, device=dev) for n in n_kp],
             "hs": [torch.empty((n, 4), dtype=torch.uint64, device=dev) for n in n_kp]}
    pidx = {c: [torch.empty((n_kp[q], 2), dtype=torch.int32, device=dev) for q, _ in w.matches] for c in plain}
    pdist = {c: [torch.empty((n_kp[q], 2), dtype=torch.uint32, device=dev) for q, _ in w.matches] for c in plain}

    def plain_pass():
        for j, im in enumerate(imgs):
            bd.build_integral(im, out=iis[j])
            bd.describe_bad(iis[j], kp_views[j], pairs, out=plain["bad"][j])
            bd.describe_hashsift(im, kp_views[j], B, t, out=plain["hs"][j])
        for c in plain:
            for m, (q, tr) in enumerate(w.matches):
                bd.match_hamming_knn(plain[c][q], plain[c][tr], k=2, idx=pidx[c][m], dist=pdist[c][m])

    ms_plain = timed(plain_pass)
    same = (torch.equal(out["bad_codes"], torch.cat(plain["bad"])) and torch.equal(out["hs_codes"], torch.cat(plain["hs"]))
            and all(torch.equal(out[f"{c}_idx"], torch.cat(pidx[c])) and torch.equal(out[f"{c}_dist"], torch.cat(pdist[c]))
                    for c in plain))
    total = b.total_kp
    pairs_n = float(sum(n_kp[q] * n_kp[tr] for q, tr in w.matches))
    b.close()
    # each stage of the batch at the roof of its binding resource (the units of
    # stage_work: HBM bytes, histogram lane-ops, MFMA operations)
    px = float(sum(im.numel() for im in imgs))
    edges = float(sum(im.shape[0] + im.shape[1] + 1 for im in imgs))
    roof = {
        "keypoint_order": roof_ms("hbm", 20.0 * total, HBM_PEAK_GBS),
        "integral": roof_ms("hbm", 5.0 * px, HBM_PEAK_GBS),
        "bad_describe": roof_ms("hbm", (16.0 + 512 / 8) * total + 4.0 * (px + edges), HBM_PEAK_GBS),
        "hashsift_features": roof_ms("alu", (1156 * 14 + 1024 * 50) * float(total), ALU_PEAK_TOPS),
        "hashsift_project": roof_ms("mfma", 2.0 * 256 * 128 * total, FP32_MFMA_PEAK_TFLOPS),
        "match_bad512": roof_ms("mfma", 2.0 * 512 * pairs_n, INT8_MFMA_PEAK_TOPS),
        "match_hashsift256": roof_ms("mfma", 2.0 * 256 * pairs_n, INT8_MFMA_PEAK_TOPS),
    }
    return {
        "workload": f"{len(imgs)} u8 images (64 scenes + shifted noisy copies), {total} keypoints, "
                    f"{sum(im.numel() for im in imgs) / 1e6:.1f} Mpx, BAD-512 + HashSIFT-256, 2-NN per scene",
        "ms_per_batch_graph": round(ms_batch, 3),
        "keypoints_per_s": round(total / (ms_batch * 1e-3), 1),
        "hamming_pairs_per_s": round(2 * pairs_n / (ms_batch * 1e-3), 1),
        "ms_per_batch_single_image_calls": round(ms_plain, 3),
        "speedup_vs_single_image_calls": round(ms_plain / ms_batch, 3),
        "roofline": {"roof_ms": round(sum(roof.values()), 4), "measured_ms": round(ms_batch, 3),
                     "frac": round(sum(roof.values()) / ms_batch, 4),
                     "roof_ms_by_stage": {k: round(v, 4) for k, v in roof.items()}},
        "bit_identical_to_single_image_calls": bool(same),
        "autotune_s": round(tune_s, 2),
        "tuning": tuning,
    }


def cpu_baseline(sample: int, runs: int = 5):
    """The oracle timed the way the paper's Table V times description: the mean
    and standard deviation of `runs` runs after one warm-up, here both on one
    core and on all host cores given to this process (at most 16, the CPU
    share of one GPU).  One run: integral images of both views, BAD-256 and
    HashSIFT-512 of `sample` keypoints per view, their 2-NN against the other
    view's full code set; scaled to the step's keypoint count.  With several
    cores the keypoint and query ranges are split over threads (the oracle's
    C calls run outside the interpreter lock); the oracle itself is the same
    single-threaded code."""
    import concurrent.futures as cf

    import oracle
    from paper_2108_08380_amd import synth

    w = synth.hashsift512_pair(synth.SEED_BASE + 1, W, H, N_KP, HS_BITS, with_bad_bits=BAD_BITS)
    oracle.lib()
    imgs_u8 = [w.extra["image1_u8"], w.extra["image2_u8"]]
    imgs_f = [w.image1, w.image2]
    kps = [w.kp1[:sample], w.kp2[:sample]]
    ii_train = oracle.build_integral(imgs_u8[1])
    bad_train = oracle.describe_bad(ii_train, w.kp2, w.pairs)[0]
    hs_train = oracle.describe_hashsift(w.image2, w.kp2, w.B, w.t)[2]
    try:
        n_all = len(os.sched_getaffinity(0))
    except AttributeError:
        n_all = os.cpu_count() or 1
    n_all = max(1, min(16, n_all))

    def one_run(pool, threads):
        cuts = np.linspace(0, sample, threads + 1).astype(int)
        parts = [(cuts[i], cuts[i + 1]) for i in range(threads) if cuts[i + 1] > cuts[i]]
        t0 = time.perf_counter()
        ii = list(pool.map(oracle.build_integral, imgs_u8))
        t_int = time.perf_counter() - t0
        t0 = time.perf_counter()
        jobs = [(v, a, b) for v in (0, 1) for a, b in parts]
        bad = list(pool.map(lambda j: oracle.describe_bad(ii[j[0]], kps[j[0]][j[1]:j[2]], w.pairs)[0], jobs))
        hs = list(pool.map(lambda j: oracle.describe_hashsift(imgs_f[j[0]], kps[j[0]][j[1]:j[2]], w.B, w.t)[2], jobs))
        t_desc = time.perf_counter() - t0
        q_bad = np.concatenate([c for (v, _, _), c in zip(jobs, bad) if v == 0])
        q_hs = np.concatenate([c for (v, _, _), c in zip(jobs, hs) if v == 0])
        t0 = time.perf_counter()
        list(pool.map(lambda ab: oracle.match_knn(q_bad[ab[0]:ab[1]], bad_train, K), parts))
        list(pool.map(lambda ab: oracle.match_knn(q_hs[ab[0]:ab[1]], hs_train, K), parts))
        t_match = time.perf_counter() - t0
        scale = N_KP / sample
        return t_int + scale * (t_desc + t_match), t_int + t_desc + t_match

    def protocol(threads):
        with cf.ThreadPoolExecutor(max_workers=threads) as pool:
            one_run(pool, threads)  # warm-up
            res = [one_run(pool, threads) for _ in range(runs)]
        rates = np.array([2 * N_KP / r[0] for r in res])
        return {"value": round(float(rates.mean()), 1), "std": round(float(rates.std()), 1),
                "step_ms_mean": round(float(np.mean([r[0] for r in res])) * 1e3, 1),
                "step_ms_std": round(float(np.std([r[0] for r in res])) * 1e3, 1),
                "seconds": round(float(sum(r[1] for r in res)), 2), "cores": threads}

    one = protocol(1)
    allc = protocol(n_all)
    return {
        "value": one["value"],
        "unit": "keypoints/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"full integral images of both views; BAD-256 + HashSIFT-512 of {sample} keypoints per view; "
                  f"{sample} queries x {N_KP} train codes 2-NN per code type; scaled to {N_KP} keypoints per view; "
                  f"mean +- std of {runs} runs after one warm-up",
        "std": one["std"],
        "runs": runs,
        "step_ms_mean": one["step_ms_mean"],
        "step_ms_std": one["step_ms_std"],
        "seconds": one["seconds"],
        "all_cores": allc,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the library has no "
                                   "multi-GPU path: each GPU would describe and match its own image pairs)"}))
        sys.exit(2)
    import torch

    dev = torch.device("cuda:0")
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb << 20
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "reps": 5}))
        return
    if args.batched_only:
        print(json.dumps({"batched_64_scenes": batched_step(dev)}))
        return
    wl = Workload(dev)
    torch.cuda.synchronize()

    # one full step first, so that a single stage run with --only reads the
    # keypoint orders, integral images and features it depends on; then the
    # warm-up (it also allocates the library workspace before any graph capture)
    wl.step()
    for _ in range(max(1, args.warmup)):
        wl.step(args.only)
    torch.cuda.synchronize()
    if args.precision_only:  # the features of the step's two views, tiled to 200000 rows
        print(json.dumps({"precision_projection_200k": precision_projection(wl)}))
        return

    graph = None
    if args.graph and not args.only:
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            wl.step()
        torch.cuda.current_stream().wait_stream(stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            wl.step()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()

    # five runs inside the timed region (events between groups of steps, no
    # extra synchronization) for the mean +- std the paper reports
    n_runs = 5 if args.steps >= 5 else 1
    marks = [args.steps * r // n_runs for r in range(n_runs + 1)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_runs + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            wl.step(args.only)
        if i + 1 in marks:
            ev[marks.index(i + 1)].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    run_ms = [ev[r].elapsed_time(ev[r + 1]) / (marks[r + 1] - marks[r]) for r in range(n_runs)]

    # the replayed graph must reproduce the eager results; also the sanity rate of
    # true matches (keypoint i of view 1 is keypoint i of view 2)
    check = {}
    if not args.only:
        snap = [x.clone() for x in (wl.bad[0], wl.hs[0], wl.idx[0], wl.idx[1])]
        wl.step()
        torch.cuda.synchronize()
        check["graph_equals_eager"] = all(torch.equal(a, b) for a, b in
                                          zip(snap, (wl.bad[0], wl.hs[0], wl.idx[0], wl.idx[1])))
        ar = torch.arange(N_KP, device=dev, dtype=torch.int32)
        check["true_match_rate_bad256"] = round(float((wl.idx[0][:, 0] == ar).float().mean()), 4)
        check["true_match_rate_hashsift512"] = round(float((wl.idx[1][:, 0] == ar).float().mean()), 4)

    stage_ms = time_stages(wl, args.stage_reps) if not args.only else {}
    work = stage_work()
    stages = {}
    step_roof = {}
    for name, (ms, ms_med, ms_min) in stage_ms.items():
        bound, units, unit = work[name][:3]
        peak = work[name][3] if len(work[name]) > 3 else peak_of(bound)
        achieved = units / (ms * 1e-3) / 1e9 if bound == "hbm" else units / (ms * 1e-3) / 1e12
        stages[name] = {"ms_per_launch": round(ms, 5), "ms_median": round(ms_med, 5), "ms_min": round(ms_min, 5),
                        "bound": bound, "achieved": round(achieved, 2),
                        "unit": unit, "peak": peak, "frac": round(achieved / peak, 4),
                        "traffic_bytes_per_launch": pmc_traffic(name)}
        step_roof[name] = roof_ms(bound, units, peak) * (2 if name in PER_VIEW_STAGES else 1)
        l1 = pmc_traffic(name, PMC_L1_ACCESSES)
        if l1 is not None:
            stages[name]["vector_l1_accesses_per_launch"] = l1
            stages[name]["vector_l1_access_frac"] = round(l1 / (ms * 1e-3) / L1_ACCESS_PEAK_PER_S, 4)
    roofline = None
    if stages:
        dom = max(stages, key=lambda n: stages[n]["ms_per_launch"])
        d = stages[dom]
        roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                    **({"vector_l1_access_frac": d["vector_l1_access_frac"]} if "vector_l1_access_frac" in d else {}),
                    "unit": d["unit"], "frac": d["frac"], "traffic": d["traffic_bytes_per_launch"],
                    "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}

    result = {
        "metric": "keypoints described/s (BAD-256, HashSIFT-512) + Hamming pairs/s, 1 MI355X",
        "value": round(2 * N_KP / (ms_per_step * 1e-3), 1),
        "unit": "keypoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u32 integer (integral, BAD); int8 MFMA with int32 sums (Hamming); f32 (HashSIFT, FP32 MFMA "
                 "projection)",
        "data": "synthetic",
        "config": {"workload": f"describe-and-match, {W}x{H} image pair, {N_KP} keypoints per view, BAD-256 + "
                               f"HashSIFT-512, Hamming 2-NN {N_KP}x{N_KP} per code type",
                   "graph": bool(graph is not None), "only": args.only or None},
        "hamming_pairs_per_s": round(2 * N_KP * N_KP / (ms_per_step * 1e-3), 1),
        "ms_per_step_5_runs": {"mean": round(float(np.mean(run_ms)), 4), "std": round(float(np.std(run_ms)), 4),
                               "steps_per_run": marks[1] - marks[0]},
        "stages": stages,
        "checks": check,
        "roofline": roofline,
    }
    if step_roof:
        # every launch of the step at the roof of its own binding resource, against the step time
        total = sum(step_roof.values())
        result["step_roofline"] = {"roof_ms": round(total, 5), "measured_ms": round(ms_per_step, 4),
                                   "frac": round(total / ms_per_step, 4),
                                   "roof_us_by_stage": {k: round(v * 1e3, 3) for k, v in step_roof.items()}}
    if not args.only and not args.step_only:
        result["describe_rates"] = describe_rates(wl)
        result["config0_bad256_640x480"] = config0_step(dev)
        result["hbm_copy"] = hbm_copy_rate(dev)
        result["same_step_via_batched_entry_point"] = pair_via_batch(wl)
        result["mutual_nn_ratio0.8"] = mutual_matching(wl)
        result["precision_projection_200k"] = precision_projection(wl)
        result["threshold_search_alg2"] = threshold_search(dev)
        result["greedy_selection_alg1"] = greedy_selection(dev)
        result["hashsift_training"] = hashsift_training(dev)
        result["differentiation_8192_triplets"] = differentiation_step(dev)
        if not args.no_batched:
            result["batched_64_scenes"] = batched_step(dev)
    if not args.no_cpu and not args.only and not args.step_only:
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
