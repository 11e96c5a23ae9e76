"""Gradient-based capacity planning over scenarios (Section 5.6 of arXiv
2410.17203): minimise, over line capacities and generator capacity
multipliers within bounds, the investment cost plus the sum over scenarios
of the planner's objective at the OPF solution, by projected gradient
descent.  Each step solves every scenario with message passing, warm-started
from that scenario's previous solution and stopped by the tolerance between
a minimum and a maximum iteration count, and takes the derivative of the
planner's objective through those unrolled iterations with the library's
adjoint.

The planner's objective is the operating cost (generator cost, battery
discharge cost, curtailment) plus an implicit per-unit penalty on each
generator's output that the OPF itself does not see (the carbon penalty of
Section 5.6).  Generator capacities scale each generator's [G][T] upper
limit profile.

The scenarios of a step are solved and differentiated in parallel on the
GPU, as the paper does (Section 5.6): each in its own context on its own
stream, driven by its own host thread (the library's calls release the
interpreter lock and capture graphs thread-locally).  Their objectives and
gradients are summed in scenario order, so the result does not depend on
which finished first.
"""
from __future__ import annotations

import copy
import dataclasses
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np

from .binding import Solver


@dataclasses.dataclass
class PlanStep:
    loss: float               # investment + sum over scenarios of the planner's objective
    operating: float          # sum over scenarios of the OPF objective
    penalty: float            # sum over scenarios of the implicit output penalty
    invest: float
    iterations: List[int]     # message-passing iterations per scenario


@dataclasses.dataclass
class PlanResult:
    line_cap: np.ndarray      # [L]
    gen_scale: np.ndarray     # [G]
    steps: List[PlanStep]


def _scenario_step(inst, cap, scale, pen, blob, dtype, eps, min_iters, max_iters,
                   checkpoint_every, opts):
    """One scenario of one step: the warm-started recorded solve, the
    planner's objective and its gradient through the adjoint, and the final
    state (the scenario's next warm start)."""
    G, T = len(inst.gen_node), int(inst.T)
    x = copy.copy(inst)
    pmax0 = np.asarray(inst.gen_pmax, float).reshape(G, T)
    x.line_cap = cap
    x.gen_pmax = pmax0 * scale[:, None]
    s = Solver(x, dtype=dtype, polish_fp64=0, eps=eps, **opts)
    try:
        if blob is not None:
            s.set_state(blob)
        res, n = s.tape_forward_warm(min_iters, max_iters, checkpoint_every)
        w = np.zeros((s.Jnc, T))
        w[:G] = pen[:, None]
        power = s.field("PNC").numpy()
        g = s.adjoint(w, 1.0)
        return dict(objective=res["objective"], penalty=float((w * power).sum()),
                    g_cap=g["cap"].cpu().numpy(), g_scale=(g["pmax"].cpu().numpy() * pmax0).sum(1),
                    blob=s.get_state(), iters=n)
    finally:
        s.close()


def plan_capacities(scenarios: Sequence, steps: int, step_size: float,
                    line_cost: np.ndarray, gen_cost: np.ndarray,
                    gen_penalty: Optional[np.ndarray] = None,
                    cap_bounds=(0.0, np.inf), scale_bounds=(0.0, np.inf),
                    min_iters: int = 250, max_iters: int = 1000, eps: float = 1e-3,
                    dtype: str = "f32", checkpoint_every: int = 50, workers: int = 4,
                    **opts) -> PlanResult:
    """Projected gradient descent on (line capacities, generator capacity
    multipliers).  scenarios: instances on the same network (same lines and
    devices; loads and generator profiles may differ).  line_cost [L] and
    gen_cost [G]: investment cost per unit of capacity (per unit of the
    multiplier for generators).  gen_penalty [G]: implicit penalty per unit
    of generator output, summed over periods.  workers: scenarios solved at
    once (1: one after another; the result is the same)."""
    base = scenarios[0]
    G = len(base.gen_node)
    cap = np.asarray(base.line_cap, float).copy()
    scale = np.ones(G)
    pen = np.zeros(G) if gen_penalty is None else np.asarray(gen_penalty, float)
    blobs: List = [None] * len(scenarios)
    history: List[PlanStep] = []
    workers = max(1, min(int(workers), len(scenarios)))
    pool = ThreadPoolExecutor(max_workers=workers) if workers > 1 else None
    try:
        for _ in range(steps + 1):
            invest = float(line_cost @ cap + gen_cost @ scale)
            g_cap = np.asarray(line_cost, float).copy()
            g_scale = np.asarray(gen_cost, float).copy()
            args = [(inst, cap, scale, pen, blobs[m], dtype, eps, min_iters, max_iters,
                     checkpoint_every, opts) for m, inst in enumerate(scenarios)]
            if pool is None:
                outs = [_scenario_step(*a) for a in args]
            else:
                outs = list(pool.map(lambda a: _scenario_step(*a), args))
            operating = penalty = 0.0
            iters = []
            for m, o in enumerate(outs):  # in scenario order
                operating += o["objective"]
                penalty += o["penalty"]
                g_cap += o["g_cap"]
                g_scale += o["g_scale"]
                blobs[m] = o["blob"]
                iters.append(o["iters"])
            history.append(PlanStep(invest + operating + penalty, operating, penalty, invest, iters))
            if len(history) > steps:
                break
            cap = np.clip(cap - step_size * g_cap, *cap_bounds)
            scale = np.clip(scale - step_size * g_scale, *scale_bounds)
    finally:
        if pool is not None:
            pool.shutdown()
    return PlanResult(cap, scale, history)
