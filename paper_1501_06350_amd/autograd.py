"""torch.autograd wrapper: x = PageRank(Z, w) with the adjoint diffusion as backward.

forward : di_init on the graph with weights w, di_diffuse(tol) -> x = H (raw result of
          x = d P x + (1-d) Z, P[i][j] = w(j->i) / s_j).
backward: di_adjoint with g = dL/dx -> dL/dZ = (1-d) lambda and dL/dw (OUT order),
          lambda = (I - d P^T)^{-1} g computed by diffusion on the transposed matrix.
All arithmetic runs in the HIP library; this module only moves tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class PageRankFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Z, w, n, out_ptr, out_idx, d, tol, tol_adj, deterministic):
        Zh = Z.detach().to("cpu", torch.float64).numpy()
        wd = None if w is None else w.detach().to(torch.float32).contiguous()
        if wd is not None and not wd.is_cuda:
            wd = wd.cuda()
        ptr = out_ptr.cuda() if not out_ptr.is_cuda else out_ptr
        idx = out_idx.cuda() if not out_idx.is_cuda else out_idx
        s = B.Solver(n, ptr.to(torch.int64).contiguous(), idx.to(torch.int32).contiguous(), wd, d=d, Z=Zh,
                     deterministic=deterministic)
        s.diffuse(tol)
        x = torch.empty(n, dtype=torch.float64, device=ptr.device)
        s.read(B.H, out=x)
        ctx.solver = s
        ctx.tol_adj = tol_adj
        ctx.has_w = w is not None
        ctx.z_device = Z.device
        ctx.z_dtype = Z.dtype
        ctx.w_device = None if w is None else w.device
        ctx.w_dtype = None if w is None else w.dtype
        return x

    @staticmethod
    def backward(ctx, gx):
        s = ctx.solver
        g = gx.detach().to(torch.float64).contiguous()
        if not g.is_cuda:
            g = g.cuda()
        # the context stays alive while the graph holds ctx (backward may run again)
        dZ, dw, _ = s.adjoint(g, ctx.tol_adj, want_dw=ctx.has_w)
        gZ = dZ.to(ctx.z_device, ctx.z_dtype)
        gw = None if dw is None else dw.to(ctx.w_device, ctx.w_dtype)
        return gZ, gw, None, None, None, None, None, None, None


def pagerank(Z, w, graph, d: float = 0.85, tol: float = 1e-12, tol_adj: float = 1e-12, deterministic: bool = False):
    """Differentiable PageRank of `graph` (object with n, out_ptr, out_idx) in Z and w."""
    ptr = torch.as_tensor(np.asarray(graph.out_ptr), dtype=torch.int64)
    idx = torch.as_tensor(np.asarray(graph.out_idx), dtype=torch.int32)
    return PageRankFn.apply(Z, w, int(graph.n), ptr, idx, float(d), float(tol), float(tol_adj), bool(deterministic))
