"""Gradients of a rollout of the step through torch.autograd.

``Rollout`` runs nsteps RK4 steps of one case (2D or 3D, any model and force)
on the GPU (the HIP step library), saving a checkpoint every ``every``
steps; its backward pass reloads the checkpoints last first and calls the
library's hand-written adjoint (tpf_step_adjoint: recompute with a tape of
stage states, then the reverse sweep) segment by segment.  Inputs with
gradients: the initial phase field phi0, the initial face velocities, the
surface tension sigma and the interface thickness eps (gradients with
respect to eps hold phi0 fixed).  This module only marshals tensors; every
step and every adjoint operator runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import tpf


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, dt, nsteps, every, sigma, eps, phi0, *u0):
        p = tpf.tpf_params()
        ctypes.memmove(ctypes.byref(p), ctypes.byref(params), ctypes.sizeof(p))
        p.sigma = float(sigma)
        p.eps = float(eps)
        p.adjoint = 1
        if len(u0) != p.dim:
            raise ValueError(f"{p.dim}D case needs {p.dim} velocity components, got {len(u0)}")
        s = tpf.Solver(p)
        dev = s.device
        # the initial state is written straight into the workspace (the views
        # round to the state's precision as tpf_set_state would)
        vphi, vu, _ = s.state_views()
        vphi.copy_(phi0.detach().reshape(s.shape))
        for a in range(p.dim):
            vu[a].copy_(u0[a].detach().reshape(s.shape))
        s.state_changed()
        ckpts = []
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            ckpts.append((s.save_checkpoint(), k))
            s.step(dt, k)
            done += k
        vphi, vu, _ = s.state_views()
        phi = vphi.to(torch.float64, copy=True)
        u = [x.to(torch.float64, copy=True) for x in vu]
        ctx.solver, ctx.ckpts, ctx.dt = s, ckpts, dt
        ctx.meta = (phi0.device, sigma.device if torch.is_tensor(sigma) else None,
                    eps.device if torch.is_tensor(eps) else None)
        return (phi.to(phi0.device),) + tuple(x.to(phi0.device) for x in u)

    @staticmethod
    def backward(ctx, gphi, *gu):
        s = ctx.solver
        dev = s.device
        g = []
        for x in (gphi,) + gu:
            g.append(torch.zeros(s.shape, dtype=torch.float64, device=dev) if x is None
                     else x.detach().to(dev, torch.float64).contiguous())
        grads = [0.0, 0.0]
        kmax = max(k for _, k in ctx.ckpts) if ctx.ckpts else 0
        tape = torch.empty(max(s.tape_bytes(kmax), 1), dtype=torch.uint8, device=dev)
        for buf, k in reversed(ctx.ckpts):
            s.load_checkpoint(buf)
            g0, gun, grads = s.step_adjoint(ctx.dt, k, g[0], g[1:], tape=tape, grad_params=grads)
            g = [g0] + list(gun)
        pdev, sdev, edev = ctx.meta
        gs = torch.tensor(grads[0], dtype=torch.float64, device=sdev or "cpu")
        ge = torch.tensor(grads[1], dtype=torch.float64, device=edev or "cpu")
        return (None, None, None, None, gs, ge) + tuple(x.to(pdev) for x in g)


def rollout(phi0, u0, sigma, eps, params, dt, nsteps, every=50):
    """phi, u after nsteps steps from (phi0, u0) with surface tension sigma and
    interface thickness eps (0-d tensors); differentiable in all four."""
    sigma = sigma if torch.is_tensor(sigma) else torch.tensor(float(sigma), dtype=torch.float64)
    eps = eps if torch.is_tensor(eps) else torch.tensor(float(eps), dtype=torch.float64)
    out = Rollout.apply(params, float(dt), int(nsteps), int(every), sigma, eps, phi0, *u0)
    return out[0], list(out[1:])
