"""torch.autograd binding of the differentiable part of the filter: the
a-trous levels (with their variance prefilter) applied to (c, var), with
gradients w.r.t. c, var and the per-level sigma_z, sigma_n, sigma_l.

Forward and backward both run in libdhr (dhr_svgf_spatial_forward,
dhr_svgf_backward); this module only marshals tensors.  The sigmas are read
to the host once per call (they parameterise the launch).
"""
from __future__ import annotations

import torch

from . import binding as B


class SVGFStack(torch.autograd.Function):
    """out = SVGFStack.apply(c, var, nz, dz, sigma_z, sigma_n, sigma_l, ctx, params)

    c, var:  float32 [F, HW] (device)      nz: [F, HW, 4]   dz: [F, HW, 2]
    sigma_*: float tensors [levels] (any device)
    ctx:     binding.Context;  params: binding.dhr_svgf_params (levels,
             eps and the rest; its sigmas are replaced by the tensors)
    W, H are taken from params-independent shapes: pass them via `shape`.
    """

    @staticmethod
    def forward(fctx, c, var, nz, dz, sigma_z, sigma_n, sigma_l, dctx, params, shape):
        W, H = shape
        F = c.shape[0]
        L = int(params.levels)
        P = _with_sigmas(params, sigma_z, sigma_n, sigma_l)
        cv = torch.stack([c.reshape(F, -1), var.reshape(F, -1)], dim=-1).to(torch.float32).contiguous()
        out = torch.empty(F, W * H, device=c.device, dtype=torch.float32)
        save = torch.empty(F, L, W * H, 2, device=c.device, dtype=torch.float32)
        nz = nz.contiguous()
        dz = dz.contiguous()
        nb = B.dhr_svgf_workspace_bytes(W, H, P, 0)
        fwork = torch.empty(F, (nb + 15) // 16 * 4, device=c.device, dtype=torch.float32)
        frames = [B.spatial_frame(W, H, cv[f], nz[f], dz[f], out[f], save=save[f], work=fwork[f]) for f in range(F)]
        B.dhr_svgf_spatial_forward(dctx, P, frames)
        fctx.save_for_backward(save, nz, dz)
        fctx.meta = (dctx, P, W, H, L, sigma_z.device)
        return out.reshape(c.shape)

    @staticmethod
    def backward(fctx, grad_out):
        save, nz, dz = fctx.saved_tensors
        dctx, P, W, H, L, sdev = fctx.meta
        F = save.shape[0]
        go = grad_out.reshape(F, W * H).to(torch.float32).contiguous()
        gcv = torch.empty(F, W * H, 2, device=go.device, dtype=torch.float32)
        nbytes = B.dhr_svgf_workspace_bytes(W, H, P, 1)
        work = torch.empty(F, (nbytes + 15) // 16 * 4, device=go.device, dtype=torch.float32)
        gs = torch.empty(3 * L, device=go.device, dtype=torch.float32)
        frames = [B.bwd_frame(W, H, save[f], nz[f], dz[f], go[f], gcv[f], work[f]) for f in range(F)]
        B.dhr_svgf_backward(dctx, P, frames, gs)
        gs = gs.to(sdev)
        return (gcv[..., 0].reshape(grad_out.shape), gcv[..., 1].reshape(grad_out.shape), None, None,
                gs[0:L], gs[L:2 * L], gs[2 * L:3 * L], None, None, None)


def _with_sigmas(params, sz, sn, sl):
    P = B.dhr_svgf_params()
    import ctypes
    ctypes.pointer(P)[0] = params
    vals = torch.stack([sz.detach(), sn.detach(), sl.detach()]).to("cpu", torch.float32).tolist()
    for l in range(int(params.levels)):
        P.sigma_z[l], P.sigma_n[l], P.sigma_l[l] = vals[0][l], vals[1][l], vals[2][l]
    return P


def svgf_stack(c, var, nz, dz, sigma_z, sigma_n, sigma_l, dctx, params, W, H):
    return SVGFStack.apply(c, var, nz, dz, sigma_z, sigma_n, sigma_l, dctx, params, (W, H))
