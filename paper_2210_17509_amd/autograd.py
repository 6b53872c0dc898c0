"""torch.autograd wrappers of the HIP step and its hand-written adjoint.

``RKSteps.apply(U, P, ctx)`` runs `steps` SSPRK steps of the HIP path, keeping
the stage checkpoints (U^n and the stage states, after con2prim) of every
step; its backward calls ``grmhd_rk_step_adjoint`` step by step in reverse.
``Con2Prim.apply(U, P_guess, ctx)`` recovers primitives; its backward is the
implicit-function-theorem VJP ``grmhd_con2prim_adjoint``.  All arithmetic runs
in libgrmhd.so.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import grmhd as G


@dataclass
class StepContext:
    dom: object
    par: object
    met: object
    dt: float
    steps: int = 1
    scheme: int = G.GRMHD_SSPRK3


def _nstage(scheme):
    return 2 if scheme == G.GRMHD_SSPRK2 else 3


class RKSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, P, sc: StepContext):
        U = U.detach().clone()
        P = P.detach().clone()
        ns = _nstage(sc.scheme)
        ck = torch.empty((sc.steps, ns) + tuple(U.shape), dtype=U.dtype, device=U.device)
        ws = None
        for k in range(sc.steps):
            ws = G.grmhd_rk_step(sc.dom, sc.par, sc.met, U, P, sc.dt, sc.scheme, ck[k], ws=ws)
        ctx.sc = sc
        ctx.save_for_backward(ck, P.detach().clone())
        ctx.mark_non_differentiable(P)
        return U, P

    @staticmethod
    def backward(ctx, gU, gP):
        sc = ctx.sc
        ck, Pfin = ctx.saved_tensors
        g_out = gU.detach().contiguous().clone()
        g_in = torch.zeros_like(g_out)
        Pw = Pfin.clone()
        ws = None
        for k in reversed(range(sc.steps)):
            ws = G.grmhd_rk_step_adjoint(sc.dom, sc.par, sc.met, ck[k], Pw, sc.dt, g_out, g_in, sc.scheme, ws=ws)
            g_out, g_in = g_in, g_out
        return g_out, None, None


class Con2Prim(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, P_guess, sc: StepContext):
        U = U.detach().clone()
        P = P_guess.detach().clone()
        G.grmhd_con2prim(sc.dom, sc.par, sc.met, U, P)
        ctx.sc = sc
        ctx.save_for_backward(P)
        return P

    @staticmethod
    def backward(ctx, gP):
        sc = ctx.sc
        (P,) = ctx.saved_tensors
        gU = torch.zeros_like(P)
        G.grmhd_con2prim_adjoint(sc.dom, sc.par, sc.met, P, gP.detach().contiguous(), gU)
        return gU, None, None
