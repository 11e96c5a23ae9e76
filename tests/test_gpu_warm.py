"""Warm start (Section 3.4) against the oracle: an iterate exported after
some iterations on one day's data, imported into the next day's network
(same structure, other loads), and run on, matches the oracle continued
from its own iterate of the same run; and the derivative of a warm-started
recorded run (the planning loop of Section 5.6) matches the oracle's
autograd through the same warm-started iterations."""
import sys

import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver as Oracle
from paper_2410_17203_amd import synth
from tests.adj_cases import tight, weights
from tests.parity import BARS, compare_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def two_days(**kw):
    args = dict(N=40, L=56, G=8, D=30, B=3, T=12, K=37, seed=21)  # two contingency chunks
    args.update(kw)
    day1 = synth.make_instance("warm", **args)
    day2 = day1.copy()
    rng = np.random.default_rng(5)
    day2.load_d = np.asarray(day1.load_d) * (1.0 + 0.03 * rng.standard_normal(day1.load_d.shape))
    return day1, day2


@pytest.mark.parametrize("dtype,adapt", [("f64", 10), ("f64", 0), ("f32", 0)])
def test_warm_started_iterates_match_oracle(dtype, adapt):
    """60 iterations on day 1 (after a penalty decision when adaptive, so a
    dual rescale is pending in the exported state), then 200 on day 2 from
    that iterate.  FP32 is compared at a fixed penalty, as for the plain
    parity runs."""
    from paper_2410_17203_amd.binding import Solver
    say(f"[warm] {dtype} adapt_every={adapt}")
    day1, day2 = two_days()
    opts = dict(rho_p=0.2, rho_theta=4.0, adapt_every=adapt)
    o1 = Oracle(day1, Options(eps=1e-12, **opts))
    o1.run(60)
    o2 = Oracle(day2, Options(eps=1e-12, **opts), init=o1.export_state())
    o2.run(200)
    a = Solver(day1, dtype=dtype, eps=1e-12, polish_fp64=0, **opts)
    a.iterate(60)
    blob = a.get_state()
    b = Solver(day2, dtype=dtype, eps=1e-12, polish_fp64=0, **opts)
    b.set_state(blob)
    b.iterate(200)
    out = compare_fields(b.field, o2.canonical_state(), BARS[dtype])
    say("  " + ", ".join(f"{k} {v[0]:.1e}/{v[1]:.1e}" for k, v in out.items()))
    gh = b.history()
    assert len(gh) == 200
    assert [(h["rho_p"], h["rho_theta"]) for h in gh] == \
        [(h.rho_p, h.rho_theta) for h in o2.history]
    if adapt:
        assert len({h.rho_p for h in o2.history}) > 1
    last = o2.history[-1]
    tol = 1e-9 if dtype == "f64" else 1e-5
    assert abs(gh[-1]["objective"] - last.objective) <= tol * abs(last.objective)
    a.close()
    b.close()


def test_warm_solve_matches_oracle_iteration_count():
    """Solve day 1, then day 2 cold and warm: in FP64 the library stops at
    the oracle's iteration in both runs, with the oracle's objective, and the
    warm run takes fewer iterations."""
    from paper_2410_17203_amd.binding import Solver
    say("[warm] solves against the oracle")
    shape = dict(synth.CONFIGS["tiny"])
    shape["K"] = 2
    day1 = synth.make_instance("warm_tiny", **shape)
    day2 = day1.copy()
    day2.load_d = np.asarray(day1.load_d) * 1.03
    opt = dict(eps=1e-3, max_iter=30000)
    o1 = Oracle(day1, Options(**opt))
    assert o1.solve().converged
    ow = Oracle(day2, Options(**opt), init=o1.export_state())
    rwo = ow.solve()
    oc = Oracle(day2, Options(**opt))
    rco = oc.solve()
    s1 = Solver(day1, dtype="f64", **opt)
    assert s1.solve()["status"] == "OPF_OK"
    blob = s1.get_state()
    warm = Solver(day2, dtype="f64", **opt)
    warm.set_state(blob)
    rw = warm.solve()
    cold = Solver(day2, dtype="f64", **opt)
    rc = cold.solve()
    say(f"  cold {rc['iter']} (oracle {rco.iter}), warm {rw['iter']} (oracle {rwo.iter})")
    assert rw["status"] == rc["status"] == "OPF_OK" and rwo.converged and rco.converged
    assert (rw["iter"], rc["iter"]) == (rwo.iter, rco.iter)
    assert abs(rw["objective"] - rwo.objective) <= 1e-9 * abs(rwo.objective)
    assert abs(rc["objective"] - rco.objective) <= 1e-9 * abs(rco.objective)
    assert rw["iter"] < rc["iter"]
    for x in (s1, warm, cold):
        x.close()


@pytest.mark.parametrize("adapt", [0, 10])
def test_warm_recorded_run_adjoint_matches_oracle(adapt):
    """opf_tape_forward_warm from an imported iterate, exactly 40 iterations,
    then opf_adjoint: the derivative of cost + <w, dispatch> with respect to
    the second day's loads, line capacities and generator limits equals the
    oracle's autograd through 40 iterations from its own iterate (the
    starting iterate is a constant of the derivative)."""
    from paper_2410_17203_amd.binding import Solver
    say(f"[warm] recorded run + adjoint, adapt_every={adapt}")
    day1 = tight("warm_adj")
    day2 = day1.copy()
    day2.load_d = np.asarray(day1.load_d) * 1.05
    opts = dict(rho_p=0.3, rho_theta=2.0, adapt_every=adapt)
    n = 40
    w = weights(day2, seed=4)
    G, T = len(day2.gen_node), int(day2.T)
    o1 = Oracle(day1, Options(eps=1e-12, **opts))
    o1.run(30)
    x = [torch.tensor(np.asarray(day2.load_d, float), requires_grad=True),
         torch.tensor(np.asarray(day2.line_cap, float), requires_grad=True),
         torch.tensor(np.asarray(day2.gen_pmax, float).reshape(G, T), requires_grad=True)]
    o2 = Oracle(day2, Options(eps=1e-12, **opts), init=o1.export_state(), load_d=x[0],
                line_cap=x[1], gen_pmax=x[2])
    o2.run(n)
    (o2.objective() + (torch.tensor(w) * o2.dispatch()).sum()).backward()
    ref = {"load": x[0].grad, "cap": x[1].grad, "pmax": x[2].grad}
    a = Solver(day1, dtype="f64", eps=1e-12, polish_fp64=0, **opts)
    a.iterate(30)
    blob = a.get_state()
    b = Solver(day2, dtype="f64", eps=1e-12, polish_fp64=0, **opts)
    b.set_state(blob)
    res, ran = b.tape_forward_warm(n, n, 10)
    assert ran == n
    g = b.adjoint(w, 1.0)
    assert float((b.field("PNC") - o2.dispatch().detach()).abs().max()) <= 1e-10 * max(
        1.0, float(o2.dispatch().detach().abs().max()))
    for k in ["load", "cap", "pmax"]:
        got, want = g[k].cpu(), ref[k]
        assert int((want != 0).sum()) > 0, k
        e = float(torch.linalg.norm(got - want)) / float(torch.linalg.norm(want))
        say(f"  {k}: relative error {e:.2e}")
        assert e <= 1e-9, (k, e)
    a.close()
    b.close()
