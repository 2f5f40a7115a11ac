"""Differentiation rule of the wave-equation operator for torch.autograd.

Mirrors the paper's rrule for F*q (section "Wave-equation-based inversion"): the forward
returns y = F(m) q and the pullback of dy is (J^T dy, F^T dy) - the gradient with respect
to the squared slowness m and with respect to the source q.  The forward keeps the
wavefield in a workspace held by the autograd context (every step when the plan stores
everything, restart slots when it checkpoints), so the pullback runs one reverse sweep
that yields both J^T dy and F^T dy.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

from .binding import STORE_NONE, Plan


class WaveOp(torch.autograd.Function):
    """d = F(m) q on a Plan; m and q are packed float32 CUDA tensors (see Plan)."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, q: torch.Tensor, plan: Plan):
        mf = m.detach().to(torch.float32).contiguous()
        qf = q.detach().to(torch.float32).contiguous()
        keep = bool(ctx.needs_input_grad[0]) and plan.storage.mode != STORE_NONE
        ws = plan.workspace(mf.device)
        d = plan.forward(mf, qf, keep=keep, ws=ws)
        ctx.plan, ctx.ws, ctx.kept = plan, ws, keep
        ctx.m_dtype = m.dtype
        ctx.save_for_backward(mf, qf)
        return d

    @staticmethod
    def backward(ctx, dy: torch.Tensor):
        mf, qf = ctx.saved_tensors
        plan = ctx.plan
        dyf = dy.detach().to(torch.float32).contiguous()
        gm = gq = None
        if ctx.needs_input_grad[0]:
            if not ctx.kept:
                raise RuntimeError("the plan keeps no wavefield (storage mode NONE): gradient "
                                   "with respect to m needs FULL or CHECKPOINT storage")
            g, v = plan.backward(mf, qf, dyf, g=True, v=bool(ctx.needs_input_grad[1]), ws=ctx.ws)
            gm = g.to(ctx.m_dtype)
            gq = v
        elif ctx.needs_input_grad[1]:
            gq = plan.adjoint(mf, dyf, ws=ctx.ws)
        ctx.ws = None
        return gm, gq, None


class BornOp(torch.autograd.Function):
    """dd = J(m, q) dm, the Born (linearised) data of a model perturbation dm about the background
    m (section "Wave-equation-based inversion": the Jacobian whose transpose gives the gradient).
    Linear in dm, so its pullback is the adjoint-state gradient J^T dy, which needs a plan with
    FULL or CHECKPOINT storage.  m and q are the fixed background; asking for their gradients is
    an error."""

    @staticmethod
    def forward(ctx, dm: torch.Tensor, m: torch.Tensor, q: torch.Tensor, plan: Plan):
        if m.requires_grad or q.requires_grad:
            raise NotImplementedError("born_forward differentiates in dm only (m and q are the background)")
        f32 = lambda t: t.detach().to(torch.float32).contiguous()
        mf, qf = f32(m), f32(q)
        ws = plan.workspace(mf.device)
        dd = plan.born(mf, qf, f32(dm), ws=ws)
        ctx.plan, ctx.ws, ctx.dm_dtype = plan, ws, dm.dtype
        ctx.save_for_backward(mf, qf)
        return dd

    @staticmethod
    def backward(ctx, dy: torch.Tensor):
        mf, qf = ctx.saved_tensors
        if ctx.plan.storage.mode == STORE_NONE:
            raise RuntimeError("the pullback of born_forward needs a plan with FULL or CHECKPOINT storage")
        g, _, _ = ctx.plan.gradient(mf, qf, dy.detach().to(torch.float32).contiguous(), ws=ctx.ws)
        ctx.ws = None
        return g.to(ctx.dm_dtype), None, None, None


def born_forward(dm: torch.Tensor, m: torch.Tensor, q: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable (in dm) Born modelling J(m, q) dm."""
    return BornOp.apply(dm, m, q, plan)


class Misfit(torch.autograd.Function):
    """phi = 1/2 ||d - d_obs||^2 on the library's residual kernel (FP64 accumulation); the
    pullback of phi is r = d - d_obs (the loss of the paper's AD listing)."""

    @staticmethod
    def forward(ctx, d: torch.Tensor, d_obs: torch.Tensor):
        from .binding import residual
        r, loss = residual(d.detach().contiguous(), d_obs.detach().contiguous())
        ctx.save_for_backward(r)
        return loss.squeeze(0)

    @staticmethod
    def backward(ctx, gphi: torch.Tensor):
        (r,) = ctx.saved_tensors
        return (r * gphi.to(r.dtype)), None


class Slowness2(torch.autograd.Function):
    """m = 1/v^2 from the compressional wavespeed v (the time-lapse operator of "Putting it all
    together" is parameterised by v); the pullback is gv = -2 gm / v^3 (library kernels)."""

    @staticmethod
    def forward(ctx, v: torch.Tensor):
        from .binding import slowness2
        vf = v.detach().to(torch.float32).contiguous()
        ctx.save_for_backward(vf)
        ctx.v_dtype = v.dtype
        return slowness2(vf)

    @staticmethod
    def backward(ctx, gm: torch.Tensor):
        from .binding import velocity_gradient
        (vf,) = ctx.saved_tensors
        return velocity_gradient(vf, gm.detach().to(torch.float32).contiguous()).to(ctx.v_dtype)


def slowness2_from_velocity(v: torch.Tensor) -> torch.Tensor:
    """Differentiable m = 1/v^2."""
    return Slowness2.apply(v)


class Patchy(torch.autograd.Function):
    """Rock physics R of "Putting it all together": (vp_new, rho_new) from the CO2 saturation
    with the rock's wavespeed, density and porosity held fixed (library kernels).  The pullback
    reaches the saturation only; asking for gradients of vp, rho or phi is an error."""

    @staticmethod
    def forward(ctx, sw, vp, rho, phi, consts):
        from .binding import patchy
        if any(t.requires_grad for t in (vp, rho, phi)):
            raise NotImplementedError("patchy_rock_physics differentiates in the saturation only")
        f32 = lambda t: t.detach().to(torch.float32).contiguous()
        args = tuple(f32(t) for t in (sw, vp, rho, phi))
        ctx.save_for_backward(*args)
        ctx.consts, ctx.sw_dtype = consts, sw.dtype
        return patchy(*args, consts=consts)

    @staticmethod
    def backward(ctx, g_vp, g_rho):
        from .binding import patchy_vjp
        sw, vp, rho, phi = ctx.saved_tensors
        f32 = lambda t: None if t is None else t.detach().to(torch.float32).contiguous()
        g_vp = torch.zeros_like(vp) if g_vp is None else f32(g_vp)
        g_sw = patchy_vjp(sw, vp, rho, phi, g_vp, f32(g_rho), consts=ctx.consts)
        return g_sw.to(ctx.sw_dtype), None, None, None, None


def patchy_rock_physics(sw, vp, rho, phi, consts=None):
    """Differentiable (in sw) patchy-saturation map: returns (vp_new, rho_new)."""
    return Patchy.apply(sw, vp, rho, phi, consts)


def misfit(d: torch.Tensor, d_obs: torch.Tensor) -> torch.Tensor:
    """Differentiable 1/2 ||d - d_obs||^2 (FP64 scalar)."""
    return Misfit.apply(d, d_obs)


def wave_forward(m: torch.Tensor, q: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable d = F(m) q."""
    return WaveOp.apply(m, q, plan)


def extend_edge(m_phys: torch.Tensor, nbl: int) -> torch.Tensor:
    """Replicate a physical-grid model nbl cells outward on every axis (differentiable; its
    backward folds the border gradient onto the edge cells)."""
    x = m_phys.unsqueeze(0).unsqueeze(0)
    pad = [nbl] * (2 * m_phys.dim())
    return F.pad(x, pad, mode="replicate")[0, 0]
