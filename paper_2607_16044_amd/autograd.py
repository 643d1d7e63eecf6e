"""torch.autograd wrappers of the engine's residual and time stepping.

* DGResidual: R^DG(U) with the hand-written vector-Jacobian product as backward.
* ARKRollout: nsteps IMEX ARK steps from U_0 (explicit-only or with an implicit
  HDG region; the facet state starts from the element traces) returning the
  states at the steps listed in ``record``.
* WallShearObjective: the wall shear of the HDG-MX region averaged over the states
  after steps n0..n1 of such a run (a scalar).
Both rollouts keep only every ``checkpoint``-th (U, Uhat) from the forward pass;
the backward pass recomputes each segment from its checkpoint and runs the step
adjoints in reverse, adding the adjoints of the recorded states (or of the
functional's terms) on the way.  Everything runs on the GPU through the C-ABI; the
tensors are FP64 device tensors in the engine's [element][variable][node] layout.
"""
from __future__ import annotations

from typing import Callable, Dict, Optional, Sequence, Tuple

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


def _clone(H):
    return None if H is None else H.clone()


def _forward_run(engine, U0, dt: float, nsteps: int, checkpoint: int,
                 visit: Callable[[int, torch.Tensor, Optional[torch.Tensor]], None]):
    """Run nsteps from U0 (facet state from the element traces), calling visit(n, U_n, H_n)
    for n = 0..nsteps; returns the checkpoints {n: (U_n, H_n)} for n = 0, c, 2c, ... < nsteps."""
    if checkpoint < 1:
        raise ValueError("checkpoint must be >= 1")
    U = U0.detach().clone().contiguous()
    H = engine.init_facets(U) if engine.sizes["n_implicit"] else None
    checkpoints = {0: (U.clone(), _clone(H))}
    visit(0, U, H)
    for n in range(1, nsteps + 1):
        engine.ark_step(dt, U, H)
        if n % checkpoint == 0 and n < nsteps:
            checkpoints[n] = (U.clone(), _clone(H))
        visit(n, U, H)
    return checkpoints, (U, H)


def _reverse(engine, dt: float, nsteps: int, every: int, checkpoints: Dict[int, Tuple], final,
             seed: Callable[[int, torch.Tensor, Optional[torch.Tensor], torch.Tensor, Optional[torch.Tensor]], None],
             duinf=None, pacc: Optional[list] = None):
    """Adjoint of U_0 for a run recorded by _forward_run.  seed(n, U_n, H_n, Ubar, Hbar)
    adds the adjoints of the state after step n into (Ubar, Hbar) in place (Hbar is None
    without an implicit region).  With duinf, pacc[0] accumulates the derivative along
    the far-field state u_inf + p duinf (U_0 fixed)."""
    U_N, H_N = final
    Ubar = torch.zeros_like(U_N)
    Hbar = None if H_N is None else torch.zeros_like(H_N)
    seed(nsteps, U_N, H_N, Ubar, Hbar)
    for c0 in sorted(checkpoints, reverse=True):
        c1 = min(c0 + every, nsteps)
        U0, H0 = checkpoints[c0]
        states = [(U0.clone(), _clone(H0))]
        for _ in range(c0, c1 - 1):
            U, H = states[-1]
            U, H = U.clone(), _clone(H)
            engine.ark_step(dt, U, H)
            states.append((U, H))
        for n in range(c1 - 1, c0 - 1, -1):
            U, H = states[n - c0]
            # the facet state seeds the Newton iterations and, for HDG-MX, the mixed
            # variables of the first explicit residual: its adjoint travels with Ubar
            Ubar, Hb = engine.vjp_imex_step(dt, U, H, Ubar.contiguous(), Hbar, return_facets=True, duinf=duinf)
            if duinf is not None:
                pacc[0] += engine.last_param_adjoint
            Hbar = Hb if Hbar is None or Hb is None else Hb.contiguous()
            seed(n, U, H, Ubar, Hbar)
    if Hbar is not None:
        # the run's first facet state is init_facets(U_0)
        Ubar = engine.vjp_init_facets(Hbar, Ubar.contiguous())
    return Ubar


class ARKRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, engine, dt: float, nsteps: int, record: Sequence[int], checkpoint: int):
        record = sorted(set(int(r) for r in record))
        if record and (record[0] < 0 or record[-1] > nsteps):
            raise ValueError("recorded steps must lie in [0, nsteps]")
        out = []

        def visit(n, U, H):
            if n in record:
                out.append(U.clone())
        ctx.checkpoints, ctx.final = _forward_run(engine, U0, dt, nsteps, checkpoint, visit)
        ctx.engine, ctx.dt, ctx.nsteps, ctx.record, ctx.every = engine, dt, nsteps, record, checkpoint
        return torch.stack(out) if out else U0.new_zeros((0,) + tuple(U0.shape))

    @staticmethod
    def backward(ctx, gout):
        seeds = {r: gout[i] for i, r in enumerate(ctx.record)}

        def seed(n, U, H, Ubar, Hbar):
            if n in seeds:
                Ubar += seeds[n]
        Ubar = _reverse(ctx.engine, ctx.dt, ctx.nsteps, ctx.every, ctx.checkpoints, ctx.final, seed)
        return Ubar, None, None, None, None, None


def ark_rollout(engine, U0, dt: float, nsteps: int, record: Sequence[int], checkpoint: int = 20):
    """States at the steps in ``record`` of an ARK run from U0, differentiable in U0."""
    return ARKRollout.apply(U0, engine, dt, nsteps, list(record), checkpoint)


class WallShearObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, p, engine, dt: float, nsteps: int, window: Tuple[int, int], checkpoint: int, duinf):
        n0, n1 = int(window[0]), int(window[1])
        if not (0 <= n0 <= n1 <= nsteps):
            raise ValueError("window must satisfy 0 <= n0 <= n1 <= nsteps")
        if engine.sizes["n_implicit"] == 0:
            raise ValueError("the wall shear is taken in the implicit HDG-MX region")
        acc = [0.0]

        def visit(n, U, H):
            if n0 <= n <= n1:
                acc[0] += engine.wall_shear(U, H)
        ctx.checkpoints, ctx.final = _forward_run(engine, U0, dt, nsteps, checkpoint, visit)
        ctx.engine, ctx.dt, ctx.nsteps, ctx.window, ctx.every = engine, dt, nsteps, (n0, n1), checkpoint
        ctx.duinf = duinf
        return U0.new_tensor(acc[0] / (n1 - n0 + 1))

    @staticmethod
    def backward(ctx, gJ):
        n0, n1 = ctx.window
        w = float(gJ) / (n1 - n0 + 1)
        eng = ctx.engine
        want_p = ctx.duinf is not None and ctx.needs_input_grad[1]

        def seed(n, U, H, Ubar, Hbar):
            if n0 <= n <= n1:
                eng.vjp_wall_shear(U, H, w, Ubar, Hbar)
        pacc = [0.0]
        Ubar = _reverse(eng, ctx.dt, ctx.nsteps, ctx.every, ctx.checkpoints, ctx.final, seed,
                        duinf=ctx.duinf if want_p else None, pacc=pacc)
        pbar = gJ.new_tensor(pacc[0]) if want_p else None
        return Ubar, pbar, None, None, None, None, None, None


def wall_shear_objective(engine, U0, dt: float, nsteps: int, window: Tuple[int, int], checkpoint: int = 20,
                         p: Optional[torch.Tensor] = None, duinf=None):
    """(1 / (n1 - n0 + 1)) sum_{n = n0}^{n1} J_wall(U_n, Uhat_n) of an ARK run from U0 (J_wall:
    the integral of mu (du/dy + dv/dx) over the HDG-MX region's walls), differentiable in U0.

    With a scalar tensor p and a direction duinf (4 floats) of the far-field state, the
    objective is also differentiable in p: the run uses the engine's far-field state, and
    the gradient of p is the derivative along u_inf + p duinf at that state (U_0 fixed).
    For the free-stream Mach number, duinf = workloads.farfield_mach_direction(...)."""
    if p is None:
        p = U0.new_zeros(())
    return WallShearObjective.apply(U0, p, engine, dt, nsteps, tuple(window), checkpoint, duinf)
