"""Reverse mode of time stepping behind torch.autograd, with checkpointing.

``rollout(stepper, u0, param, nsteps, every, dstate)`` advances ``u0`` by
``nsteps`` calls of fcsd_step and returns the final state.  Its backward is
the hand-written discrete adjoint (fcsd_step_adj) with the decisions of the
forward run frozen (network classes, step sizes; the derivative of the
branch that was taken, like the reverse mode of any piecewise map):

  * forward: the state is kept every ``every`` steps (checkpoints); each
    step's classes (int8 plane) and step size are recorded;
  * backward: segments are processed last to first; a segment is re-run
    from its checkpoint with the recorded decisions (fcsd_step replay,
    bit-identical to the forward run) writing a step record per step (its
    glued stage inputs, viscosity, maximisers, pre-filter state and the FC
    derivatives of the stage inputs that the reverse mode uses), then
    reversed step by step from the records, so no step is run forward a
    third time.  With ``record=False`` the replay keeps only each step's
    input and fcsd_step_adj recomputes the step from it.

Memory: nsteps/every checkpoints + ``every`` step records (66 planes each;
4 with record=False) + one int8 plane and one float per step, instead of
all nsteps states.

``param`` is a scalar tensor on which only the Dirichlet boundary state
depends inside the stepping (e.g. the inflow Mach number); ``dstate`` is
d(boundary state)/d(param) (4 floats).  Its gradient is accumulated by the
glue transposes.  Dependence of the initial state on parameters is left to
torch (build u0 from them with torch operations).
"""
from __future__ import annotations

import torch

from .api import Stepper


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, param, stepper: Stepper, nsteps: int, every: int, dstate, record: bool):
        st = stepper
        st.u.copy_(u0)
        ckpts, taus, dts = {}, [], []
        for n in range(nsteps):
            if n % every == 0:
                ckpts[n] = st.u.clone()
            st.step()
            taus.append(st.tau.clone())
            dts.append(st.dt.clone())
        ctx.stepper, ctx.ckpts, ctx.taus, ctx.dts = st, ckpts, taus, dts
        ctx.nsteps, ctx.every, ctx.dstate = nsteps, every, tuple(float(v) for v in dstate)
        ctx.record = record
        return st.u.clone()

    @staticmethod
    def backward(ctx, u_bar):
        st = ctx.stepper
        ub = u_bar.contiguous().clone()
        dparam = torch.zeros(1, dtype=torch.float64, device=ub.device)
        recs = [st.new_record() for _ in range(min(ctx.every, ctx.nsteps))] if ctx.record else None
        for seg0 in reversed(range(0, ctx.nsteps, ctx.every)):
            seg1 = min(seg0 + ctx.every, ctx.nsteps)
            st.u.copy_(ctx.ckpts[seg0])
            inputs = []
            for n in range(seg0, seg1):
                if recs is None:
                    inputs.append(st.u.clone())
                st.replay(ctx.taus[n], ctx.dts[n], record=recs[n - seg0] if recs else None)
            for n in reversed(range(seg0, seg1)):
                if recs is None:
                    st.step_adj(inputs[n - seg0], ub, ctx.taus[n], ctx.dts[n], ctx.dstate, dparam)
                else:
                    st.step_adj(None, ub, ctx.taus[n], ctx.dts[n], ctx.dstate, dparam, record=recs[n - seg0])
        return ub, dparam.to(torch.float32).reshape(()), None, None, None, None, None


def rollout(stepper: Stepper, u0: torch.Tensor, param: torch.Tensor, nsteps: int, every: int = 8,
            dstate=(0.0, 0.0, 0.0, 0.0), record: bool = True) -> torch.Tensor:
    """Final state after nsteps steps of `stepper` from u0 (differentiable in
    u0 and param; see the module docstring)."""
    return _Rollout.apply(u0, param, stepper, int(nsteps), int(every), dstate, bool(record))


def freestream_dmach(mach: float, gamma: float = 1.4):
    """d/dM of the inflow state (rho, rho u, rho v, E) = (1.4, 1.4 M, 0,
    1/(gamma-1) + 0.7 M^2) of the annulus workloads."""
    return (0.0, 1.4, 0.0, 1.4 * float(mach))
