"""Differentiable multi-step rollout of the time step (torch.autograd.Function).

forward:  u_K = S_{K-1}( ... S_0(u_0)) with each step's dt from the CFL rule on
          the device; the state is kept every `every` steps (checkpoints) and
          each step's (dt, c_h) is recorded.  The steps of the last segment
          write their tapes and keep their input states already (the backward
          pass starts there, so they need no recomputation).
backward: for each checkpoint segment, last first: recompute the segment's
          states from its checkpoint with the recorded dt, each step writing
          its tape (switches and face traces), then apply lwfr_adjoint_step
          with those tapes from the last step of the segment to the first.
          The gradient is that of the step sequence with dt, c_h, alpha, the
          thetas and every max/abs branch frozen at their forward values.

All arithmetic runs in the HIP library; torch holds the buffers and the
autograd bookkeeping.
"""
import torch

from . import lwfr


class LwfrRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, stepper, nsteps, every):
        if not (stepper.cfg.flags & lwfr.LWFR_CFG_ADJOINT):
            raise ValueError("the stepper's configuration needs LWFR_CFG_ADJOINT for the backward pass")
        if nsteps < 1 or every < 1:
            raise ValueError("nsteps and every must be positive")
        dtch = torch.zeros((nsteps, 2), dtype=torch.float64, device=u0.device)
        ua = u0.detach().contiguous().clone()
        ub = torch.empty_like(ua)
        ckpts = []
        last0 = (nsteps - 1) // every * every  # first step of the last segment
        tapes = [stepper.new_tape() for _ in range(min(every, nsteps))]
        last_states = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(ua.clone())
            if n >= last0:
                # the same step (dt from the device), also writing its tape
                last_states.append(ua.clone())
                stepper.step_taped(ua, ub, 0.0, tapes[n - last0], dtch[n])
            else:
                stepper.step(ua, ub, 0.0, dtch[n])
            ua, ub = ub, ua
        ctx.stepper, ctx.nsteps, ctx.every = stepper, nsteps, every
        ctx.tapes, ctx.last_states = tapes, last_states
        ctx.save_for_backward(dtch, *ckpts)
        return ua

    @staticmethod
    def backward(ctx, grad):
        dtch, *ckpts = ctx.saved_tensors
        st, K, k = ctx.stepper, ctx.nsteps, ctx.every
        dts = dtch[:, 0].tolist()
        lam = grad.contiguous().clone()
        out = torch.empty_like(lam)
        tapes = ctx.tapes
        for seg in reversed(range(len(ckpts))):
            n0, n1 = seg * k, min(seg * k + k, K)
            if seg == len(ckpts) - 1:
                states = ctx.last_states  # taped in the forward pass
            else:
                states = [ckpts[seg]]
                for n in range(n0, n1):
                    nxt = torch.empty_like(lam)
                    st.step_taped(states[-1], nxt, dts[n], tapes[n - n0])
                    states.append(nxt)
            for n in reversed(range(n0, n1)):
                st.adjoint_step(states[n - n0], dts[n], lam, out, tapes[n - n0])
                lam, out = out, lam
        ctx.tapes = ctx.last_states = None
        return lam, None, None, None


def rollout(u0, stepper, nsteps, every=5):
    """u after `nsteps` steps from u0, differentiable w.r.t. u0 (checkpoint every `every` steps)."""
    return LwfrRollout.apply(u0, stepper, nsteps, every)


def replay(u0, stepper, dtch):
    """The step sequence with each step's dt and c_h taken from dtch (n x 2), no autograd."""
    ua = u0.contiguous().clone()
    ub = torch.empty_like(ua)
    vals = dtch.tolist()
    for dt, ch in vals:
        stepper.step_fixed(ua, ub, dt, ch)
        ua, ub = ub, ua
    return ua
