"""Differentiable unrolled RSKA: K multi-RHS steps as a torch.autograd.Function.

The forward runs the float32 MFMA multi-RHS solve and keeps x* checkpoints
every ``ckpt_every`` steps; the backward is the hand-written adjoint
(rsk_avg_adjoint), which recomputes each segment from its checkpoint and
returns gradients with respect to B, lambda and the per-step relaxations
alpha_k. A, the index stream and eta are not differentiated.
"""
from __future__ import annotations

import torch

from . import rsk


class RSKAvgUnrolled(torch.autograd.Function):
    """X_K = RSKAvgUnrolled.apply(B, lam, alpha_k, A, index_stream, eta, ckpt_every, rownorm2).

    B: m x R float32 (R a multiple of 4); lam: 0-dim tensor; alpha_k: K float32
    (K = len(alpha_k)); A: m x n float32; index_stream: K*eta int32. Returns
    x_K = S_lambda(x*_K) (n x R). The subgradient of S_lambda is 1[|x*| > lambda].
    """

    @staticmethod
    def forward(ctx, B, lam, alpha_k, A, index_stream, eta, ckpt_every, rownorm2_t=None):
        K = int(alpha_k.numel())
        n, R = A.shape[1], B.shape[1]
        r2 = rownorm2_t if rownorm2_t is not None else rsk.rownorm2(A)
        nseg = max(1, -(-K // ckpt_every))
        ckpt = torch.empty((nseg, n, R), dtype=A.dtype, device=A.device)
        lam_f = float(lam)
        Bc = B.detach().contiguous()
        ak = alpha_k.detach().contiguous()
        res = rsk.solve_multirhs(A, Bc, lam=lam_f, eta=eta, alpha=1.0, K=K, index_stream=index_stream,
                                 alpha_k=ak, rownorm2_t=r2, ckpt=ckpt, ckpt_every=ckpt_every)
        ctx.save_for_backward(Bc, ak, res.x_star, ckpt, r2)
        ctx.A, ctx.index_stream, ctx.eta, ctx.ckpt_every, ctx.lam = A, index_stream, eta, ckpt_every, lam_f
        ctx.lam_shape = lam.shape if torch.is_tensor(lam) else ()
        ctx.lam_dtype = lam.dtype if torch.is_tensor(lam) else torch.float32
        return res.x

    @staticmethod
    def backward(ctx, gX):
        Bc, ak, x_star_K, ckpt, r2 = ctx.saved_tensors
        adj = rsk.adjoint_multirhs(ctx.A, Bc, lam=ctx.lam, eta=ctx.eta, alpha_k=ak, K=int(ak.numel()),
                                   index_stream=ctx.index_stream, ckpt=ckpt, ckpt_every=ctx.ckpt_every,
                                   X_star_K=x_star_K, Xbar_K=gX.detach().contiguous(), rownorm2_t=r2)
        lam_bar = adj.lambda_bar.to(ctx.lam_dtype).reshape(ctx.lam_shape)
        return adj.Bbar, lam_bar, adj.alpha_bar, None, None, None, None, None


def rska_unrolled(B, lam, alpha_k, A, index_stream, eta, ckpt_every=20, rownorm2_t=None):
    """Functional form of RSKAvgUnrolled."""
    return RSKAvgUnrolled.apply(B, lam, alpha_k, A, index_stream, eta, ckpt_every, rownorm2_t)
