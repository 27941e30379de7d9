"""torch.autograd.Function over the C ABI: resistance distances as a
differentiable function of the edge weights.

forward(w): writes the weights into the graph handle (rd_set_weights) and
runs the batched Lanczos iteration (rd_query_batch) for the pairs.
backward(g): rd_grad_edges, which re-runs the iteration and accumulates the
potentials phi = L^+ (e_s - e_t) (estimated as in Algorithm 5) to form
dL/dw_e = -sum_p g_p (phi_p(u) - phi_p(v))^2.

This is the derivative of the exact r(s,t) evaluated at the Lanczos
potentials, not the derivative of the truncated Lanczos estimate.
Only marshalling happens here; every step runs in the HIP library.
"""

from __future__ import annotations

import torch

from . import rd


def _opts(precision: int, stream: int, **kw) -> rd.RdOptions:
    o = rd.rd_default_options(precision=precision, stream=stream, **kw)
    o.flags |= rd.RD_DEVICE_PTRS
    return o


class ResistanceDistance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w: torch.Tensor, graph: "rd.RDGraph", s: torch.Tensor, t: torch.Tensor,
                eps: float = 1e-6, precision: int = rd.RD_F64, block_width: int = 0):
        if not (w.is_cuda and s.is_cuda and t.is_cuda):
            raise ValueError("weights and pair lists must be CUDA tensors")
        wd = w.detach().contiguous()
        graph.set_weights(wd)
        stream = torch.cuda.current_stream().cuda_stream
        out = torch.empty(s.numel() * 24, dtype=torch.uint8, device=w.device)
        graph.query_batch(s.contiguous(), t.contiguous(), eps,
                          _opts(precision, stream, block_width=block_width), out=out)
        r = out.view(torch.float64).view(-1, 3)[:, 0].clone()
        ctx.graph = graph
        ctx.eps = eps
        ctx.precision = precision
        ctx.block_width = block_width
        ctx.save_for_backward(wd, s, t)
        return r

    @staticmethod
    def backward(ctx, grad_r: torch.Tensor):
        wd, s, t = ctx.saved_tensors
        graph = ctx.graph
        graph.set_weights(wd)  # the handle may have seen other weights since forward
        stream = torch.cuda.current_stream().cuda_stream
        gw = torch.empty(graph.m, dtype=torch.float32, device=wd.device)
        graph.grad_edges(s.contiguous(), t.contiguous(), grad_r.detach().double().contiguous(), ctx.eps,
                         _opts(ctx.precision, stream, block_width=ctx.block_width), fwd=None,
                         grad_w=gw)
        return gw.to(wd.dtype), None, None, None, None, None, None


def resistance_distance(w: torch.Tensor, graph: "rd.RDGraph", s: torch.Tensor, t: torch.Tensor,
                        eps: float = 1e-6, precision: int = rd.RD_F64, block_width: int = 0):
    """r(s_p, t_p) for every pair, differentiable in the edge weights w
    (aligned with the edge list the graph was built from)."""
    return ResistanceDistance.apply(w, graph, s, t, eps, precision, block_width)
