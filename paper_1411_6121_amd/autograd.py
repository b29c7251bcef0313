"""Differentiable DUGKS rollout: torch.autograd.Function over the library's
forward step, hand-written adjoint step, initial-state VJP and read-out VJP,
with sqrt(N) checkpointing (Griewank-style two-level recomputation).

Memory: ceil(sqrt(N)) checkpoint states plus one segment of at most
ceil(sqrt(N)) states during the backward pass; compute: one extra forward
pass.  Any mesh and boundary set of the incompressible model (those of the
adjoint step).
"""
from __future__ import annotations

import math

import torch

from . import (dugks_destroy, dugks_init, dugks_init_vjp, dugks_moments, dugks_moments_vjp, dugks_reset,
               dugks_step, dugks_step_adjoint, shape_of, torch_dtype)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(actx, force, u0, cfg, nsteps, seg):
        Q, D, shp = shape_of(cfg)
        dt = float(cfg["dt"])
        f = torch.empty((Q,) + shp, dtype=force.dtype, device=force.device)
        g = torch.empty_like(f)
        h = dugks_init(cfg, f, None, u0, force)
        ckpt = {0: f.clone()}
        for n in range(nsteps):
            dugks_step(h, f, g, force, n * dt)
            f, g = g, f
            if (n + 1) % seg == 0 and (n + 1) < nsteps:
                ckpt[n + 1] = f.clone()
        u = torch.empty((D,) + shp, dtype=force.dtype, device=force.device)
        dugks_moments(h, f, force, nsteps * dt, None, u, None, totals=False)
        actx.h, actx.cfg, actx.nsteps, actx.seg, actx.ckpt = h, cfg, nsteps, seg, ckpt
        actx.save_for_backward(force, u0)
        return u

    @staticmethod
    def backward(actx, grad_u):
        force, u0 = actx.saved_tensors
        h, cfg, nsteps, seg, ckpt = actx.h, actx.cfg, actx.nsteps, actx.seg, actx.ckpt
        dt = float(cfg["dt"])
        Q, D, shp = shape_of(cfg)
        grad_u = grad_u.contiguous()
        gforce = torch.zeros_like(force)
        lam = torch.empty((Q,) + shp, dtype=force.dtype, device=force.device)
        lam2 = torch.empty_like(lam)
        dugks_moments_vjp(h, lam, None, grad_u, nsteps * dt, gforce)
        starts = sorted(ckpt.keys())
        # one segment's states, recomputed step by step straight into their
        # slots (slot 0 is the checkpoint itself)
        seg_states = torch.empty((seg - 1, Q) + shp, dtype=force.dtype, device=force.device) if seg > 1 else None
        for s0 in reversed(starts):
            s1 = min(s0 + seg, nsteps)

            def state(n):
                return ckpt[s0] if n == s0 else seg_states[n - s0 - 1]

            for n in range(s0, s1 - 1):
                dugks_step(h, state(n), state(n + 1), force, n * dt)
            for n in reversed(range(s0, s1)):
                dugks_step_adjoint(h, state(n), lam, lam2, force, n * dt, gforce)
                lam, lam2 = lam2, lam
        gu0 = torch.zeros_like(u0)
        dugks_init_vjp(h, lam, u0, force, 0.0, gu0, gforce)
        dugks_destroy(h)
        actx.h = None
        return gforce, gu0, None, None, None


def rollout(cfg: dict, force: torch.Tensor, u0: torch.Tensor, nsteps: int, segment: int | None = None):
    """Final velocity u(t_N) [D, nz, ny, nx] after nsteps from the equilibrium
    state at (rho0, u0) under the force field `force`; differentiable in
    force and u0."""
    seg = segment or max(1, math.ceil(math.sqrt(nsteps)))
    return _Rollout.apply(force.contiguous(), u0.contiguous(), dict(cfg), int(nsteps), int(seg))
