"""Differentiation of a trajectory through the hand-written discrete adjoint.

``advance_fixed_dt(cfg, U0, nsteps, dt, every)`` advances U0 by nsteps
TVD-RK3 steps at a fixed time step and is differentiable with
torch.autograd: the backward pass is the reverse sweep of the library's
``rk3_step_adjoint`` (vector-Jacobian products of the fused right-hand side,
Sec. 3.2, and of the Runge-Kutta stages, Sec. 3.4), the derivative the paper
obtains by automatic differentiation of its solver (Sec. 6).

Memory: the forward pass keeps one state every ``every`` steps (checkpoints);
the backward pass recomputes one segment at a time from its checkpoint, stage by
stage (``rk3_stage``), keeping every step's state and its two stage states, and
sweeps it in reverse with ``rk3_step_adjoint_stages`` (the stage states are not
recomputed), so at most 3 ``every`` + nsteps/every states are held.  The time step is a constant of the trajectory (not
differentiated).  Coverage is that of rk3_step_adjoint: single-phase Euler,
FP64, limiters off.

``kinetic_energy`` is the loss of the gradient check.
"""
from __future__ import annotations

import torch

from . import solver as S


# Workspaces of the forward and reverse sweeps, kept per (workspace size, device) and
# reused by later calls on problems of the same size (the tensors are only scratch:
# every call overwrites them before reading).  Trajectories differentiated at the
# same time on one device (several streams or threads) would share them: run them
# one after another.
_WS: dict = {}


def _scratch(kind: str, nbytes: int, device) -> torch.Tensor:
    key = (kind, int(nbytes), str(device))
    t = _WS.get(key)
    if t is None:
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        _WS[key] = t
    return t


def _segment_states(every: int, like: torch.Tensor) -> torch.Tensor:
    """Buffer for the recomputed states of one checkpoint segment (reused): for each
    step its state U^n and its stage states U^(1), U^(2)."""
    key = ("segment", every, tuple(like.shape), like.dtype, str(like.device))
    t = _WS.get(key)
    if t is None:
        t = torch.empty((every, 3) + tuple(like.shape), dtype=like.dtype, device=like.device)
        _WS[key] = t
    return t


class _Advance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, cfg, nsteps, dt, every):
        U = U0.detach().clone().contiguous()
        ws = _scratch("ws", S.workspace_bytes(cfg), U.device)
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(U.clone())
            S.rk3_step(cfg, U, dt, ws)
        ctx.save_for_backward(*ckpts)
        ctx.cfg, ctx.nsteps, ctx.dt, ctx.every = cfg, nsteps, dt, every
        return U

    @staticmethod
    def backward(ctx, Ubar):
        cfg, nsteps, dt, every = ctx.cfg, ctx.nsteps, ctx.dt, ctx.every
        ckpts = ctx.saved_tensors
        G = Ubar.detach().clone().contiguous()
        aws = _scratch("aws", S.adjoint_workspace_bytes(cfg), G.device)
        states = _segment_states(every, G)
        for seg in range(len(ckpts) - 1, -1, -1):
            first = seg * every
            count = min(every, nsteps - first)
            # the segment recomputed stage by stage from its checkpoint (the same stage
            # kernels as rk3_step): U^n, U^(1), U^(2) of every step
            states[0, 0].copy_(ckpts[seg])
            for n in range(count):
                Un, U1, U2 = states[n, 0], states[n, 1], states[n, 2]
                S.rk3_stage(cfg, 1, Un, Un, U1, dt)
                S.rk3_stage(cfg, 2, Un, U1, U2, dt)
                if n + 1 < count:
                    S.rk3_stage(cfg, 3, Un, U2, states[n + 1, 0], dt)
            for n in range(count - 1, -1, -1):
                S.rk3_step_adjoint_stages(cfg, states[n, 0], states[n, 1], states[n, 2], G, dt, aws)
        return G, None, None, None, None


def advance_fixed_dt(cfg: S.Config, U0: torch.Tensor, nsteps: int, dt: float, every: int = 10) -> torch.Tensor:
    """U(nsteps) from U0 at a fixed dt; differentiable in U0 (checkpoint every ``every`` steps)."""
    if every < 1:
        raise ValueError("every must be >= 1")
    return _Advance.apply(U0, cfg, int(nsteps), float(dt), int(every))


def kinetic_energy(cfg: S.Config, U: torch.Tensor) -> torch.Tensor:
    """Volume-integrated kinetic energy sum 1/2 |rho u|^2 / rho dV."""
    rho = U[0]
    mom2 = U[1] ** 2 + U[2] ** 2 + U[3] ** 2
    return 0.5 * (mom2 / rho).sum() * (cfg.dx * cfg.dy * cfg.dz)
