"""torch.autograd.Function wrappers of the differentiation entry points.

Each forward and backward is a single call into the library's kernels
(bd_relaxed_*_fwd/bwd, bd_trl_hnm_fwd/bwd); these classes only save the
tensors the backward kernels need.  Gradients flow to the relaxed BAD
parameters (box weights w1, w2 and thresholds theta), to the HashSIFT
projection (B, t) and through the triplet ranking loss to the descriptors;
patches and features are treated as constants.
"""
from __future__ import annotations

import torch

import paper_2108_08380_amd as bd


class RelaxedBAD(torch.autograd.Function):
    """D = tanh(beta * (theta - (w1 * m1 - w2 * m2))) per patch and pair."""

    @staticmethod
    def forward(ctx, patches, w1, w2, theta, pairs, beta: float):
        D, m1, m2 = bd.relaxed_bad_fwd(patches, pairs, w1.contiguous(), w2.contiguous(), theta.contiguous(), beta)
        ctx.save_for_backward(D, m1, m2)
        ctx.beta = beta
        return D

    @staticmethod
    def backward(ctx, gD):
        D, m1, m2 = ctx.saved_tensors
        g_w1, g_w2, g_theta = bd.relaxed_bad_bwd(gD.contiguous(), D, m1, m2, ctx.beta)
        return None, g_w1, g_w2, g_theta, None, None


class RelaxedHashSIFT(torch.autograd.Function):
    """D = tanh(beta * (B f - t)) for precomputed features f."""

    @staticmethod
    def forward(ctx, f, B, t, beta: float):
        _, D = bd.relaxed_hashsift_fwd(f, B.contiguous(), t.contiguous(), beta)
        ctx.save_for_backward(D, f)
        ctx.beta = beta
        return D

    @staticmethod
    def backward(ctx, gD):
        D, f = ctx.saved_tensors
        gB, gt = bd.relaxed_hashsift_bwd(gD.contiguous(), D, f, ctx.beta)
        return None, gB, gt, None


class TripletHNMLoss(torch.autograd.Function):
    """mean_i [tau - s(a_i, p_i) + s_neg(i)]_+ with in-batch hardest negatives and anchor swap."""

    @staticmethod
    def forward(ctx, A, P, tau: float):
        A, P = A.contiguous(), P.contiguous()
        loss, neg, hinge = bd.trl_hnm_fwd(A, P, tau)
        ctx.save_for_backward(A, P, neg, hinge)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        A, P, neg, hinge = ctx.saved_tensors
        gA, gP = bd.trl_hnm_bwd(A, P, neg, hinge, g.reshape(1).to(torch.float32))
        return gA, gP, None


def bad_triplet_loss(anchor, positive, w1, w2, theta, pairs, beta: float = 10.0, tau: float = 0.5):
    """Training loss of relaxed BAD codes over a batch of (anchor, positive) patches."""
    return TripletHNMLoss.apply(RelaxedBAD.apply(anchor, w1, w2, theta, pairs, beta),
                                RelaxedBAD.apply(positive, w1, w2, theta, pairs, beta), tau)


def hashsift_triplet_loss(f_anchor, f_positive, B, t, beta: float = 10.0, tau: float = 0.5):
    """Training loss of relaxed HashSIFT codes over precomputed patch features."""
    return TripletHNMLoss.apply(RelaxedHashSIFT.apply(f_anchor, B, t, beta),
                                RelaxedHashSIFT.apply(f_positive, B, t, beta), tau)
