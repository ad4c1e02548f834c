"""Differentiable point-to-point registration loss over the dilation NNS.

``P2PLoss`` wraps the forward and backward kernels of libvicp in a
``torch.autograd.Function``.  For pair b with pose xi_b = (rho, phi):

    L_b = (1/m_b) sum_i |Exp(xi_b) p_i - q_c(i)|^2     (Eq. 1 per point)

with c(i) found by the local/global voxel search at the float32-rounded pose.
Correspondences are held fixed when differentiating and are recomputed in
the backward pass rather than stored.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, lib
from .api import Grid, _i64, _ptrs, _stream

__all__ = ["P2PLoss", "p2p_loss"]


class P2PLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p_soa: torch.Tensor, xi: torch.Tensor, grid: Grid, m_per_pair):
        B = grid.npairs
        if xi.shape != (B, 6) or xi.dtype != torch.float64 or not xi.is_cuda:
            raise ValueError("xi must be a (npairs, 6) float64 CUDA tensor")
        p_soa = p_soa.contiguous()
        xi = xi.contiguous()
        loss = torch.empty(B, dtype=torch.float64, device=p_soa.device)
        px, py, pz = _ptrs(p_soa)
        check(lib().vicp_p2p_loss_fwd(grid.handle, px, py, pz, _i64(m_per_pair), C.c_void_p(xi.data_ptr()),
                                      C.c_void_p(loss.data_ptr()), _stream()), "vicp_p2p_loss_fwd")
        ctx.save_for_backward(p_soa, xi)
        ctx.grid = grid
        ctx.m = list(m_per_pair)
        return loss

    @staticmethod
    def backward(ctx, gloss: torch.Tensor):
        p_soa, xi = ctx.saved_tensors
        gloss = gloss.to(torch.float64).contiguous()
        dp = torch.empty_like(p_soa)
        dxi = torch.empty_like(xi)
        px, py, pz = _ptrs(p_soa)
        dx, dy, dz = _ptrs(dp)
        check(lib().vicp_p2p_loss_bwd(ctx.grid.handle, px, py, pz, _i64(ctx.m), C.c_void_p(xi.data_ptr()),
                                      C.c_void_p(gloss.data_ptr()), dx, dy, dz, C.c_void_p(dxi.data_ptr()),
                                      _stream()), "vicp_p2p_loss_bwd")
        return dp, dxi, None, None


def p2p_loss(grid: Grid, p: torch.Tensor, xi: torch.Tensor, m_per_pair=None) -> torch.Tensor:
    """Per-pair loss (B,) float64.

    ``p`` is (B, m, 3) (equal sizes) or SoA (3, sum m) float32 CUDA; ``xi`` is
    (B, 6) float64 CUDA.  Both may require grad.
    """
    B = grid.npairs
    if p.dim() == 3:
        if p.shape[0] != B or p.shape[2] != 3:
            raise ValueError("p must be (npairs, m, 3)")
        m_per_pair = [p.shape[1]] * B
        p_soa = p.permute(2, 0, 1).reshape(3, -1)
    else:
        if p.shape[0] != 3:
            raise ValueError("p must be (3, sum m) in SoA layout")
        p_soa = p
        if m_per_pair is None:
            if B != 1:
                raise ValueError("m_per_pair is required for a batched grid")
            m_per_pair = [p.shape[1]]
    if p_soa.dtype != torch.float32 or not p_soa.is_cuda:
        raise TypeError("p must be float32 CUDA")
    return P2PLoss.apply(p_soa, xi, grid, list(m_per_pair))
