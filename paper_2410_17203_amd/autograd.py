"""PyTorch autograd over unrolled message-passing iterations.

`unrolled_dispatch` runs a fixed number of iterations on the GPU from the zero
start (Section 4.4 of arXiv 2410.17203: the iterate after n steps is a
composition of almost-everywhere differentiable maps of the problem data) and
returns the device powers and the objective of the last iterate.  Its
backward pass is the library's hand-written adjoint (`opf_adjoint`): no
graph of the iterations is recorded by PyTorch, only checkpoints of the
iterate, and the penalty schedule of the forward run is held fixed.

Differentiable inputs: load demand [D, T], line capacities [L], generator
upper limits [G, T].  Everything else comes from the instance.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from .binding import Solver


def _with_data(inst, load_d, line_cap, gen_pmax):
    out = copy.copy(inst)
    out.load_d = load_d.detach().cpu().double().numpy().reshape(np.shape(inst.load_d))
    out.line_cap = line_cap.detach().cpu().double().numpy().reshape(np.shape(inst.line_cap))
    out.gen_pmax = gen_pmax.detach().cpu().double().numpy().reshape(np.shape(inst.gen_pmax))
    return out


class _Unrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, load_d, line_cap, gen_pmax, inst, n_iters, checkpoint_every, dtype, opts):
        solver = Solver(_with_data(inst, load_d, line_cap, gen_pmax), dtype=dtype,
                        polish_fp64=0, **opts)
        res = solver.tape_forward(n_iters, checkpoint_every)
        power = solver.field_device("PNC").clone()
        obj = torch.tensor(res["objective"], dtype=torch.float64, device=power.device)
        ctx.solver = solver
        # each gradient goes back on its input's device, in its dtype and shape
        ctx.like = [(x.shape, x.dtype, x.device) for x in (load_d, line_cap, gen_pmax)]
        return power, obj

    @staticmethod
    def backward(ctx, g_power, g_obj):
        solver = ctx.solver
        if solver is None:
            raise RuntimeError("unrolled_dispatch: backward ran twice; the recorded run is "
                               "released after the first backward (retain_graph is not supported)")
        cot = None if g_power is None else g_power.to(solver.device, torch.float64).contiguous()
        w = 0.0 if g_obj is None else float(g_obj)
        grads = solver.adjoint(cot, w)
        solver.close()
        ctx.solver = None
        out = [grads[k].reshape(shape).to(device=dev, dtype=dt)
               for k, (shape, dt, dev) in zip(("load", "cap", "pmax"), ctx.like)]
        return (*out, None, None, None, None, None)


def unrolled_dispatch(inst, load_d: torch.Tensor, line_cap: torch.Tensor,
                      gen_pmax: torch.Tensor, n_iters: int, checkpoint_every: int = 50,
                      dtype: str = "f64", **opts):
    """Device powers [G+D+B, T] and objective after n_iters iterations, with
    gradients w.r.t. load_d, line_cap and gen_pmax through the library's
    adjoint.  opts map onto opf_options (penalties, adaptive rule, inner
    iterations)."""
    return _Unrolled.apply(load_d, line_cap, gen_pmax, inst, int(n_iters), int(checkpoint_every),
                           dtype, dict(opts))
