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
"""
from __future__ import annotations

import copy
import dataclasses
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


def plan_capacities(scenarios: Sequence, steps: int, step_size: float,
                    line_cost: np.ndarray, gen_cost: np.ndarray,
                    gen_penalty: Optional[np.ndarray] = None,
                    cap_bounds=(0.0, np.inf), scale_bounds=(0.0, np.inf),
                    min_iters: int = 250, max_iters: int = 1000, eps: float = 1e-3,
                    dtype: str = "f32", checkpoint_every: int = 50, **opts) -> PlanResult:
    """Projected gradient descent on (line capacities, generator capacity
    multipliers).  scenarios: instances on the same network (same lines and
    devices; loads and generator profiles may differ).  line_cost [L] and
    gen_cost [G]: investment cost per unit of capacity (per unit of the
    multiplier for generators).  gen_penalty [G]: implicit penalty per unit
    of generator output, summed over periods."""
    base = scenarios[0]
    L, G = len(base.line_from), len(base.gen_node)
    cap = np.asarray(base.line_cap, float).copy()
    scale = np.ones(G)
    pen = np.zeros(G) if gen_penalty is None else np.asarray(gen_penalty, float)
    blobs: List = [None] * len(scenarios)
    history: List[PlanStep] = []
    for _ in range(steps + 1):
        invest = float(line_cost @ cap + gen_cost @ scale)
        g_cap = np.asarray(line_cost, float).copy()
        g_scale = np.asarray(gen_cost, float).copy()
        operating = penalty = 0.0
        iters = []
        for m, inst in enumerate(scenarios):
            x = copy.copy(inst)
            T = int(inst.T)
            pmax0 = np.asarray(inst.gen_pmax, float).reshape(G, T)
            x.line_cap = cap
            x.gen_pmax = pmax0 * scale[:, None]
            s = Solver(x, dtype=dtype, polish_fp64=0, eps=eps, **opts)
            if blobs[m] is not None:
                s.set_state(blobs[m])
            res, n = s.tape_forward_warm(min_iters, max_iters, checkpoint_every)
            J = s.Jnc
            w = np.zeros((J, T))
            w[:G] = pen[:, None]
            power = s.field("PNC").numpy()
            operating += res["objective"]
            penalty += float((w * power).sum())
            g = s.adjoint(w, 1.0)
            g_cap += g["cap"].cpu().numpy()
            g_scale += (g["pmax"].cpu().numpy() * pmax0).sum(1)
            blobs[m] = s.get_state()
            s.close()
            iters.append(n)
        history.append(PlanStep(invest + operating + penalty, operating, penalty, invest, iters))
        if len(history) > steps:
            break
        cap = np.clip(cap - step_size * g_cap, *cap_bounds)
        scale = np.clip(scale - step_size * g_scale, *scale_bounds)
    return PlanResult(cap, scale, history)
