"""Differentiable grid integration: torch.autograd.Function wrappers whose
backward passes are the library's own adjoint kernels.

rho(D, tau, eps): the density of Eq. 3 for density matrix D at atom positions
tau under a homogeneous strain eps (positions and cell mapped by 1 + eps, the
fractional grid fixed).  With a cotangent g on rho, L = sum_g g_g rho_g and

    dL/dD     = H[V := g / w]                (gint_vlocal: Vlocal is the adjoint of rho)
    dL/dtau   = -F[V := g / w] (1 + eps)     (gint_force_stress, Eq. 4)
    dL/deps   = Z[V := g / w] (1 + eps)^-T   (gint_force_stress, Eq. 5 strain derivative)

because E = sum_g w V_g rho_g equals L when V = g / w.  energy(V, D, tau,
eps) = w0 sum_g V_g rho_g (w0 the unstrained volume per point) has
dE/dV = w0 rho, dE/dD = H[V], dE/dtau = -F (1 + eps), dE/deps = Z (1 + eps)^-T.

A plan (neighbour lists) is built for the geometry of a forward call and
reused by later calls with the same system, positions, strain and precision
(an SCF loop calls rho at fixed geometry); its host build time is kept in
`last_plan_seconds`.  Plans are released when the last autograd context
holding them goes away, not in backward, so backward can run more than once
(retain_graph).  Every numeric step runs in the HIP library; the energy is
the library's FP64 reduction w sum_g V_g rho_g (gint_energy).
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import gint as G


_plan_cache = {}
last_plan_seconds = 0.0


def _plan_for(system, tau: torch.Tensor, eps: torch.Tensor, precision: int):
    """Plan of the strained geometry; one cached entry, reused while the
    system, positions, strain and precision are the same."""
    global last_plan_seconds
    s, M = _geometry(system, tau, eps)
    key = (id(system), precision, s.pos.tobytes(), s.cell.tobytes())
    hit = _plan_cache.get("entry")
    if hit is not None and hit[0] == key and hit[1] is system:
        return hit[2], M
    plan = G.Plan(s, precision=precision)
    last_plan_seconds = float(plan.sizes.build_seconds)
    _plan_cache["entry"] = (key, system, plan)
    return plan, M


def _geometry(system, tau: torch.Tensor, eps: torch.Tensor):
    s = copy.copy(system)
    M = np.eye(3) + eps.detach().cpu().numpy().astype(np.float64)
    s.pos = np.ascontiguousarray(tau.detach().cpu().numpy().astype(np.float64) @ M.T)
    s.cell = np.ascontiguousarray(np.asarray(system.cell, dtype=np.float64) @ M.T)
    return s, M


def _adjoints(plan, v_like: torch.Tensor, d: torch.Tensor, need_d: bool, need_geo: bool):
    dev = v_like.device
    out = {}
    if need_d:
        h = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
        G.gint_vlocal(plan, v_like, h)
        out["D"] = h
    if need_geo:
        F = torch.empty(3 * plan.natom, dtype=torch.float64, device=dev)
        sig = torch.empty(9, dtype=torch.float64, device=dev)
        G.gint_force_stress(plan, v_like, d, F, sig)
        out["F"] = F.view(-1, 3)
        out["Z"] = -sig.view(3, 3) * plan.volume
    return out


class GintRho(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d, tau, eps, system, precision):
        plan, M = _plan_for(system, tau, eps, precision)
        rho = torch.empty(plan.ngrid, dtype=torch.float64, device=d.device)
        G.gint_rho(plan, d.contiguous(), rho)
        ctx.plan = plan
        ctx.M = M
        ctx.save_for_backward(d)
        return rho

    @staticmethod
    def backward(ctx, gbar):
        (d,) = ctx.saved_tensors
        plan = ctx.plan
        w = plan.volume / plan.ngrid
        v_like = (gbar.contiguous() / w).to(torch.float64)
        need_d = ctx.needs_input_grad[0]
        need_geo = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        adj = _adjoints(plan, v_like, d.contiguous(), need_d, need_geo)
        gd = adj.get("D")
        Mt = torch.tensor(ctx.M, dtype=torch.float64, device=gbar.device)
        # positions are M tau, so dL/dtau = (dL/dpos) M
        gtau = -adj["F"] @ Mt if need_geo and ctx.needs_input_grad[1] else None
        geps = None
        if need_geo and ctx.needs_input_grad[2]:
            minv_t = torch.tensor(np.linalg.inv(ctx.M).T, dtype=torch.float64, device=gbar.device)
            geps = adj["Z"] @ minv_t
        return gd, gtau, geps, None, None


class GintEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, d, tau, eps, system, precision):
        plan, M = _plan_for(system, tau, eps, precision)
        rho = torch.empty(plan.ngrid, dtype=torch.float64, device=d.device)
        G.gint_rho(plan, d.contiguous(), rho)
        w0 = float(abs(np.linalg.det(np.asarray(system.cell, dtype=np.float64)))) / plan.ngrid
        # the plan's w is the strained w0 det(M); V rescaled so that w V = w0 V
        scale = w0 / (plan.volume / plan.ngrid)
        e = torch.empty(1, dtype=torch.float64, device=d.device)
        G.gint_energy(plan, (v.to(torch.float64) * scale).contiguous(), rho, e)
        e = e[0]
        ctx.plan, ctx.M, ctx.w0 = plan, M, w0
        ctx.save_for_backward(v, d, rho)
        return e

    @staticmethod
    def backward(ctx, ebar):
        v, d, rho = ctx.saved_tensors
        plan = ctx.plan
        # the kernels use the strained w = w0 det(M); rescale V so that w V = w0 V
        scale = ctx.w0 / (plan.volume / plan.ngrid)
        v_like = (v.to(torch.float64) * scale).contiguous()
        need_d = ctx.needs_input_grad[1]
        need_geo = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        adj = _adjoints(plan, v_like, d.contiguous(), need_d, need_geo)
        gv = ebar * ctx.w0 * rho if ctx.needs_input_grad[0] else None
        gd = ebar * adj["D"] if need_d else None
        Mt = torch.tensor(ctx.M, dtype=torch.float64, device=ebar.device)
        gtau = -ebar * (adj["F"] @ Mt) if need_geo and ctx.needs_input_grad[2] else None
        geps = None
        if need_geo and ctx.needs_input_grad[3]:
            minv_t = torch.tensor(np.linalg.inv(ctx.M).T, dtype=torch.float64, device=ebar.device)
            geps = ebar * (adj["Z"] @ minv_t)
        return gv, gd, gtau, geps, None, None


def rho(system, d, tau=None, eps=None, precision: int = G.GINT_FP64):
    """Differentiable density of `system` (inputs.System-like) on cuda tensors."""
    dev = d.device
    if tau is None:
        tau = torch.tensor(system.pos, dtype=torch.float64, device=dev)
    if eps is None:
        eps = torch.zeros(3, 3, dtype=torch.float64, device=dev)
    return GintRho.apply(d, tau, eps, system, precision)


def energy(system, v, d, tau=None, eps=None, precision: int = G.GINT_FP64):
    """Differentiable E = w0 sum_g V_g rho_g."""
    dev = d.device
    if tau is None:
        tau = torch.tensor(system.pos, dtype=torch.float64, device=dev)
    if eps is None:
        eps = torch.zeros(3, 3, dtype=torch.float64, device=dev)
    return GintEnergy.apply(v, d, tau, eps, system, precision)
