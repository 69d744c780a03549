"""torch.autograd bindings of the library's hand-written adjoint.

ResidualFn   R = residual(w); backward calls fdu_residual_vjp.
RKUnroll     w_N = N SSP-RK3 steps at a fixed dt from w_0; the forward keeps a
             state every ``ckpt_every`` steps and the stage states of the last
             segment's steps; the backward recomputes each earlier segment from
             its checkpoint stage by stage, keeping every step's stage states,
             and applies fdu_rk_step_vjp_stages in reverse (no stage state is
             computed more than once per pass).

Every forward and backward pass runs in the HIP library; these classes only
hold tensors and order the calls.
"""
from __future__ import annotations

import torch


class ResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, solver):
        w_in = w.detach().contiguous()              # read only: the library fills ghost rows in a copy
        R = solver.residual(w_in)
        ctx.save_for_backward(w_in)
        ctx.solver = solver
        return R

    @staticmethod
    def backward(ctx, Rbar):
        (w_in,) = ctx.saved_tensors
        wbar = ctx.solver.residual_vjp(w_in, Rbar.contiguous())
        return wbar, None


class RKUnroll(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w0, solver, nsteps: int, dt: float, ckpt_every: int = 5):
        dev = w0.device
        w = w0.detach().contiguous().clone()
        scratch = torch.empty(2 * solver.nv_total, 4, dtype=w.dtype, device=dev)
        dt_dev = torch.full((1,), float(dt), dtype=torch.float64, device=dev)
        ckpts = [w.clone()]
        # the last segment's steps run stage by stage and keep their stage
        # states: the backward starts there and need not recompute them
        last_start = ((nsteps - 1) // ckpt_every) * ckpt_every if nsteps > 0 else 0
        tail = []
        for i in range(nsteps):
            if i >= last_start:
                wn, w1, w2 = w.clone(), torch.empty_like(w), torch.empty_like(w)
                solver.rk_stage(0, wn, wn, w1, dt_dev)
                solver.rk_stage(1, wn, w1, w2, dt_dev)
                solver.rk_stage(2, wn, w2, w, dt_dev)
                tail += [wn, w1, w2]
            else:
                solver.rk_step(w, scratch, dt_dev)
            if (i + 1) % ckpt_every == 0 and i + 1 < nsteps:
                ckpts.append(w.clone())
        ctx.solver, ctx.nsteps, ctx.dt, ctx.ckpt_every = solver, nsteps, float(dt), ckpt_every
        ctx.n_ckpts = len(ckpts)
        ctx.save_for_backward(*ckpts, *tail)
        return w

    @staticmethod
    def backward(ctx, wbar):
        solver, nsteps, dt, every = ctx.solver, ctx.nsteps, ctx.dt, ctx.ckpt_every
        saved_all = ctx.saved_tensors
        ckpts, tail = saved_all[:ctx.n_ckpts], saved_all[ctx.n_ckpts:]
        dev = wbar.device
        dt_dev = torch.full((1,), dt, dtype=torch.float64, device=dev)
        scratch2 = torch.empty(2 * solver.nv_total, 4, dtype=wbar.dtype, device=dev)
        g = wbar.contiguous().clone()
        g[solver.nv_real:] = 0.0
        gn = torch.empty_like(g)
        for seg in reversed(range(len(ckpts))):
            start = seg * every
            stop = min(start + every, nsteps)
            if seg == len(ckpts) - 1:
                # the last segment's stage states, kept by the forward pass
                saved = [tuple(tail[3 * j:3 * j + 3]) for j in range(stop - start)]
            else:
                # recompute the segment stage by stage, keeping every step's
                # stage states (the step adjoints then need no forward
                # recompute of their own; the last step needs only its first
                # two stages)
                saved = []
                wn = ckpts[seg].clone()
                for i in range(start, stop):
                    w1, w2 = torch.empty_like(wn), torch.empty_like(wn)
                    solver.rk_stage(0, wn, wn, w1, dt_dev)
                    solver.rk_stage(1, wn, w1, w2, dt_dev)
                    saved.append((wn, w1, w2))
                    if i + 1 < stop:
                        wnext = torch.empty_like(wn)
                        solver.rk_stage(2, wn, w2, wnext, dt_dev)
                        wn = wnext
            for j in reversed(range(stop - start)):
                solver.rk_step_vjp_stages(*saved[j], g, gn, scratch2, dt)
                g, gn = gn, g
        return g, None, None, None, None


def residual(solver, w):
    return ResidualFn.apply(w, solver)


def rk_unroll(solver, w0, nsteps: int, dt: float, ckpt_every: int = 5):
    return RKUnroll.apply(w0, solver, nsteps, dt, ckpt_every)
