"""torch.autograd wrappers of the engine's residual and time stepping.

* DGResidual: R^DG(U) with the hand-written vector-Jacobian product as backward.
* ARKRollout: nsteps IMEX ARK steps from U_0 (explicit-only or with an implicit
  HDG region; the facet state starts from the element traces) returning the
  states at the steps listed in ``record``; the backward pass keeps only every
  ``checkpoint``-th (U, Uhat) from the forward pass and recomputes each segment
  from its checkpoint, then runs the step adjoints in reverse, adding the
  adjoints of the recorded states on the way (so time-averaged functionals of
  the trajectory are differentiable).
Both run entirely on the GPU through the C-ABI; the tensors are FP64 device
tensors in the engine's [element][variable][node] layout.
"""
from __future__ import annotations

from typing import Sequence

import torch


class DGResidual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, engine):
        ctx.engine = engine
        ctx.save_for_backward(U)
        return engine.dg_residual(U.contiguous())

    @staticmethod
    def backward(ctx, Rbar):
        (U,) = ctx.saved_tensors
        return ctx.engine.vjp_dg_residual(U.contiguous(), Rbar.contiguous()), None


def dg_residual(engine, U):
    return DGResidual.apply(U, engine)


class ARKRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, engine, dt: float, nsteps: int, record: Sequence[int], checkpoint: int):
        if checkpoint < 1:
            raise ValueError("checkpoint must be >= 1")
        record = sorted(set(int(r) for r in record))
        if record and (record[0] < 0 or record[-1] > nsteps):
            raise ValueError("recorded steps must lie in [0, nsteps]")
        U = U0.detach().clone().contiguous()
        H = engine.init_facets(U) if engine.sizes["n_implicit"] else None
        checkpoints = {0: (U.clone(), None if H is None else H.clone())}
        out = []
        if 0 in record:
            out.append(U.clone())
        for n in range(1, nsteps + 1):
            engine.ark_step(dt, U, H)
            if n % checkpoint == 0 and n < nsteps:
                checkpoints[n] = (U.clone(), None if H is None else H.clone())
            if n in record:
                out.append(U.clone())
        ctx.engine, ctx.dt, ctx.nsteps, ctx.record, ctx.every = engine, dt, nsteps, record, checkpoint
        ctx.checkpoints = checkpoints
        return torch.stack(out) if out else U.new_zeros((0,) + tuple(U.shape))

    @staticmethod
    def backward(ctx, gout):
        eng, dt, nsteps, every = ctx.engine, ctx.dt, ctx.nsteps, ctx.every
        seed = {r: gout[i] for i, r in enumerate(ctx.record)}
        Ubar = torch.zeros_like(ctx.checkpoints[0][0])
        Hbar = None
        if nsteps in seed:
            Ubar += seed[nsteps]
        starts = sorted(ctx.checkpoints)
        for c0 in reversed(starts):
            c1 = min(c0 + every, nsteps)
            # recompute the states (U, Uhat)_{c0} .. (U, Uhat)_{c1-1} of this segment
            U0, H0 = ctx.checkpoints[c0]
            states = [(U0.clone(), None if H0 is None else H0.clone())]
            for _ in range(c0, c1 - 1):
                U, H = states[-1]
                U, H = U.clone(), None if H is None else H.clone()
                eng.ark_step(dt, U, H)
                states.append((U, H))
            for n in range(c1 - 1, c0 - 1, -1):
                U, H = states[n - c0]
                # the facet state seeds the Newton iterations and, for HDG-MX, the mixed
                # variables of the first explicit residual: its adjoint travels with Ubar
                Ubar, Hbar = eng.vjp_imex_step(dt, U, H, Ubar.contiguous(), Hbar, return_facets=True)
                if n in seed:
                    Ubar += seed[n]
        if Hbar is not None:
            # the run's first facet state is init_facets(U_0)
            Ubar = eng.vjp_init_facets(Hbar, Ubar.contiguous())
        return Ubar, None, None, None, None, None


def ark_rollout(engine, U0, dt: float, nsteps: int, record: Sequence[int], checkpoint: int = 20):
    """States at the steps in ``record`` of an ARK run from U0, differentiable in U0."""
    return ARKRollout.apply(U0, engine, dt, nsteps, list(record), checkpoint)
