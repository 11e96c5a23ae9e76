"""Gradient-based capacity planning (Section 5.6): projected gradient steps
on line capacities and generator capacity multipliers, each step solving the
scenarios with warm-started message passing and differentiating through the
unrolled iterations with the library's adjoint."""
import sys

import numpy as np
import pytest

from paper_2410_17203_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def scenarios(n=2):
    """The 14-node grid with halved line capacities and curtailable loads (so
    every capacity choice is feasible), two load scenarios."""
    out = []
    for m in range(n):
        inst = synth.config("tiny")
        rng = np.random.default_rng(100 + m)
        inst.load_d = np.asarray(inst.load_d) * rng.uniform(0.9, 1.2, np.shape(inst.load_d))
        inst.line_cap = np.asarray(inst.line_cap) * 0.5
        out.append(synth.with_curtailable_loads(inst, cost=60.0))
    return out


def plan(sc, steps, **kw):
    """Costs and bounds of the 14-node planning case."""
    from paper_2410_17203_amd.planning import plan_capacities
    L, G = len(sc[0].line_from), len(sc[0].gen_node)
    G0 = G - len(synth.config("tiny").load_node)  # real generators; the rest are loads
    free = np.zeros(G - G0)
    return plan_capacities(
        sc, steps=steps, step_size=3e-3, line_cost=np.full(L, 2.0),
        gen_cost=np.r_[np.full(G0, 1.0), free],
        gen_penalty=np.r_[np.where(np.arange(G0) % 2 == 0, 10.0, 0.0), free],
        cap_bounds=(0.0, 10.0),
        scale_bounds=(np.r_[np.full(G0, 0.3), free + 1.0], np.r_[np.full(G0, 3.0), free + 1.0]),
        min_iters=250, max_iters=20000, eps=1e-4, dtype="f64", **kw), G0


def test_planning_lowers_the_planner_loss():
    say("[planning] 8 gradient steps, 2 scenarios")
    r, G0 = plan(scenarios(), 8)
    losses = [s.loss for s in r.steps]
    say("  losses " + " ".join(f"{x:.2f}" for x in losses))
    say("  iterations " + str([s.iterations for s in r.steps]))
    assert len(r.steps) == 9
    # every solve stopped by the tolerance, after at least the minimum
    assert all(250 <= n < 20000 for s in r.steps for n in s.iterations)
    assert losses[-1] < losses[0] - 0.1 * abs(losses[0])
    assert np.all(r.line_cap >= 0.0) and np.all(r.line_cap <= 10.0)
    assert np.all(r.gen_scale[G0:] == 1.0)  # loads are not resized


def test_concurrent_scenarios_give_the_sequential_result():
    # each scenario in its own context, stream and host thread: the same
    # solves, and the objectives and gradients summed in scenario order
    say("[planning] 3 steps, 4 scenarios, one after another and four at once")
    sc = scenarios(4)
    r1, _ = plan(sc, 3, workers=1)
    r4, _ = plan(sc, 3, workers=4)
    assert [s.iterations for s in r1.steps] == [s.iterations for s in r4.steps]
    assert [s.loss for s in r1.steps] == [s.loss for s in r4.steps]
    assert np.array_equal(r1.line_cap, r4.line_cap)
    assert np.array_equal(r1.gen_scale, r4.gen_scale)
