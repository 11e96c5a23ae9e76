"""Hand-written adjoint of unrolled iterations (Section 4.4) against the
oracle's autograd derivative (pinned by finite differences in
test_oracle_grad.py), against finite differences of the GPU forward at the
differentiation workload, and for consistency (checkpoint interval, FP32 vs
FP64, the autograd wrapper)."""
import copy
import sys

import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver as Oracle
from paper_2410_17203_amd import synth
from tests.adj_cases import tight, weights

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = torch.as_tensor(a, dtype=torch.float64).cpu()
    b = torch.as_tensor(b, dtype=torch.float64).cpu()
    nb = float(torch.linalg.norm(b))
    return float(torch.linalg.norm(a - b)) / max(nb, 1e-300)


def oracle_grads(inst, n_iters, w, w_obj, **opt):
    G, T = len(inst.gen_node), int(inst.T)
    x = [torch.tensor(np.asarray(inst.load_d, float), requires_grad=True),
         torch.tensor(np.asarray(inst.line_cap, float), requires_grad=True),
         torch.tensor(np.asarray(inst.gen_pmax, float).reshape(G, T), requires_grad=True)]
    o = Oracle(inst, Options(eps=1e-12, **opt), load_d=x[0], line_cap=x[1], gen_pmax=x[2])
    o.run(n_iters)
    f = w_obj * o.objective() + (torch.tensor(w) * o.dispatch()).sum()
    f.backward()
    return {"load": x[0].grad, "cap": x[1].grad, "pmax": x[2].grad}, o


def gpu_grads(inst, n_iters, w, w_obj, dtype="f64", every=50, **opt):
    from paper_2410_17203_amd.binding import Solver
    s = Solver(inst, dtype=dtype, polish_fp64=0, **opt)
    res = s.tape_forward(n_iters, every)
    g = s.adjoint(w, w_obj)
    out = {k: v.cpu() for k, v in g.items()}
    power = s.field("PNC")
    s.close()
    return out, res, power


CASES = {
    "fixed_penalty": dict(adapt_every=0, rho_p=0.3, rho_theta=2.0),
    "adaptive_penalty": dict(adapt_every=10, rho_p=0.3, rho_theta=2.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_adjoint_matches_oracle_autograd(case):
    say(f"[adjoint] fp64 vs oracle autograd, {case}")
    opt = CASES[case]
    inst = tight()
    w = weights(inst)
    ref, o = oracle_grads(inst, 60, w, 1.0, **opt)
    got, res, power = gpu_grads(inst, 60, w, 1.0, **opt)
    assert res["iter"] == 60
    last = o.history[-1]  # penalties used by the last iteration
    assert (res["rho_p"], res["rho_theta"]) == (last.rho_p, last.rho_theta)
    assert rel(power, o.dispatch().detach()) <= 1e-10
    for k in ["load", "cap", "pmax"]:
        assert int((ref[k] != 0).sum()) > 0, k  # clips of every kind were active
        e = rel(got[k], ref[k])
        say(f"  {k}: relative error {e:.2e}")
        assert e <= 1e-9, (k, e)


@pytest.mark.parametrize("shape", [dict(T=1, K=0, B=0), dict(T=1, K=4, B=2), dict(T=70, K=2, B=3),
                                   dict(T=24, K=6, B=0, G=6)])
def test_fp64_adjoint_other_shapes(shape):
    say(f"[adjoint] fp64 shape {shape}")
    kw = dict(N=12, L=17, G=4, D=8, seed=5)
    kw.update(shape)
    inst = tight("adj_shape", **kw)
    w = weights(inst, seed=3)
    opt = dict(adapt_every=10, rho_p=0.5, rho_theta=1.0)
    ref, _ = oracle_grads(inst, 50, w, 0.5, **opt)
    got, _, _ = gpu_grads(inst, 50, w, 0.5, **opt)
    for k in ["load", "cap", "pmax"]:
        if got[k].numel():
            assert rel(got[k], ref[k]) <= 1e-9, (k, rel(got[k], ref[k]))


def test_checkpoint_interval_does_not_change_the_result():
    say("[adjoint] checkpoint intervals")
    inst = tight()
    w = weights(inst)
    opt = CASES["adaptive_penalty"]
    outs = [gpu_grads(inst, 60, w, 1.0, every=e, **opt)[0] for e in (1, 7, 60, 100)]
    for o in outs[1:]:
        for k in o:
            assert torch.equal(o[k], outs[0][k]), k


def test_fp32_adjoint_close_to_fp64():
    say("[adjoint] fp32 vs fp64")
    inst = tight()
    w = weights(inst)
    opt = CASES["adaptive_penalty"]
    g64, _, _ = gpu_grads(inst, 60, w, 1.0, dtype="f64", **opt)
    g32, _, _ = gpu_grads(inst, 60, w, 1.0, dtype="f32", **opt)
    for k in g64:
        e = rel(g32[k], g64[k])
        say(f"  {k}: fp32 relative error {e:.2e}")
        assert e <= 1e-3, (k, e)


def general_case(name):
    """The derivative test grid with the general line model (Section 2.3):
    DC links with tight capacities (contingency 1 takes the first link out),
    per-contingency changes (second outages, ratings, susceptances), or both
    (changes then also reach the links)."""
    base = tight("adj_gen", N=16, L=24, G=4, D=10, B=2, T=6, K=6, seed=81)
    if name in ("hvdc", "both"):
        base = synth.with_dc_links(base, 3, seed=5, cap=(0.1, 0.3))
    if name in ("changes", "both"):
        base = synth.with_contingency_changes(base, seed=6, second_outages=2, rating_changes=8,
                                              sus_changes=3)
    return base


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("name", ["hvdc", "changes", "both"])
def test_fp64_adjoint_general_line_model_matches_oracle_autograd(name, case):
    say(f"[adjoint] fp64 vs oracle autograd, general line model {name}, {case}")
    inst = general_case(name)
    w = weights(inst, seed=4)
    opt = CASES[case]
    ref, o = oracle_grads(inst, 60, w, 1.0, **opt)
    got, res, power = gpu_grads(inst, 60, w, 1.0, **opt)
    assert rel(power, o.dispatch().detach()) <= 1e-10
    for k in ["load", "cap", "pmax"]:
        e = rel(got[k], ref[k])
        say(f"  {k}: relative error {e:.2e} ({int((ref[k] != 0).sum())} nonzero)")
        assert e <= 1e-9, (k, e)
    # line clips were active (this grid's generators stay below their limits)
    assert int((ref["load"] != 0).sum()) > 0 and int((ref["cap"] != 0).sum()) > 0
    if name != "changes":  # some DC link capacity clipped its flow
        dc = np.nonzero(np.asarray(inst.line_kind) == 1)[0]
        assert float(ref["cap"][dc].abs().sum()) > 0.0


def test_general_line_model_adjoint_checkpoints_and_fp32():
    say("[adjoint] general line model: checkpoint intervals, fp32 vs fp64")
    inst = general_case("both")
    w = weights(inst, seed=4)
    opt = CASES["adaptive_penalty"]
    outs = [gpu_grads(inst, 60, w, 1.0, every=e, **opt)[0] for e in (1, 7, 60)]
    for o in outs[1:]:
        for k in o:
            assert torch.equal(o[k], outs[0][k]), k
    g32, _, _ = gpu_grads(inst, 60, w, 1.0, dtype="f32", **opt)
    for k in outs[0]:
        e = rel(g32[k], outs[0][k])
        say(f"  {k}: fp32 relative error {e:.2e}")
        assert e <= 1e-3, (k, e)


def test_autograd_function_gives_the_adjoint():
    from paper_2410_17203_amd.autograd import unrolled_dispatch
    say("[adjoint] autograd wrapper")
    inst = tight()
    w = torch.tensor(weights(inst), device="cuda")
    G, T = len(inst.gen_node), int(inst.T)
    scale = torch.ones(len(inst.load_node), dtype=torch.float64, device="cuda", requires_grad=True)
    d0 = torch.tensor(np.asarray(inst.load_d, float), device="cuda")
    cap = torch.tensor(np.asarray(inst.line_cap, float), device="cuda", requires_grad=True)
    pmax = torch.tensor(np.asarray(inst.gen_pmax, float).reshape(G, T), device="cuda",
                        requires_grad=True)
    opt = CASES["adaptive_penalty"]
    power, obj = unrolled_dispatch(inst, scale[:, None] * d0, cap, pmax, 60, 20, **opt)
    (obj + (w * power).sum()).backward()
    ref, _ = oracle_grads(inst, 60, weights(inst), 1.0, **opt)
    assert rel(scale.grad, (ref["load"] * torch.tensor(np.asarray(inst.load_d))).sum(1)) <= 1e-9
    assert rel(cap.grad, ref["cap"]) <= 1e-9
    assert rel(pmax.grad, ref["pmax"]) <= 1e-9
    # CPU inputs: gradients come back on the CPU, in the inputs' dtype; a
    # second backward through the released run is a clear error
    x = [torch.tensor(np.asarray(inst.load_d, float), requires_grad=True),
         cap.detach().cpu().float().requires_grad_(),
         pmax.detach().cpu().requires_grad_()]
    power, obj = unrolled_dispatch(inst, x[0], x[1], x[2], 60, 20, **opt)
    loss = obj + (w * power).sum()
    loss.backward(retain_graph=True)
    assert x[0].grad.device.type == "cpu" and x[1].grad.dtype == torch.float32
    assert rel(x[0].grad, ref["load"]) <= 1e-9 and rel(x[2].grad, ref["pmax"]) <= 1e-9
    with pytest.raises(RuntimeError, match="backward ran twice"):
        loss.backward()


def _diff_forward(inst, scale, cap, n_iters, dtype="f64"):
    """Objective and <w, power> after n_iters at the given load scales and
    capacities (GPU forward only)."""
    from paper_2410_17203_amd.binding import Solver
    x = copy.copy(inst)
    x.load_d = np.asarray(inst.load_d) * scale[:, None]
    x.line_cap = cap
    s = Solver(x, dtype=dtype, polish_fp64=0, eps=0.0, min_iter=2**31 - 1, max_iter=2**31 - 1)
    s.iterate(n_iters)
    r = s.residuals()
    p = s.field("PNC").numpy()
    s.close()
    return r, p


def test_diff_workload_against_finite_differences():
    """Differentiation workload (500 nodes, 700 lines, T = 24, K = 20), 1000
    unrolled iterations with checkpoints every 50: derivatives of the cost
    and of <w, dispatch> w.r.t. the 400 load scale factors and 700 line
    capacities against central differences of the FP64 GPU forward at 20
    seed-chosen coordinates, and directional derivatives along 8 random
    directions."""
    from paper_2410_17203_amd.binding import Solver
    say("[adjoint] diff workload, 1000 iterations")
    inst = synth.config("diff")
    n_iters = 1000
    D, L = len(inst.load_node), len(inst.line_from)
    w = weights(inst, seed=2024)
    s = Solver(inst, dtype="f64", polish_fp64=0)
    res = s.tape_forward(n_iters, 50)
    g = s.adjoint(w, 1.0)
    s.close()
    d0 = np.asarray(inst.load_d)
    g_scale = (g["load"].cpu().numpy() * d0).sum(1)
    g_cap = g["cap"].cpu().numpy()
    say(f"  nonzero cap derivatives: {int((g_cap != 0).sum())} of {L}")

    def f(scale, cap):
        r, p = _diff_forward(inst, scale, cap, n_iters)
        return r["objective"] + float((w * p).sum()), r

    one, cap0 = np.ones(D), np.asarray(inst.line_cap, float)
    r0 = f(one, cap0)[1]
    assert abs(r0["objective"] - res["objective"]) <= 1e-12 * abs(res["objective"])
    rng = np.random.default_rng(2024)
    # small enough that few of the ~1e8 clip evaluations switch inside +-h,
    # large enough that FP64 rounding of f (~1e4) stays near 1e-5 absolute
    h = 1e-6
    errs = []
    for q in rng.choice(D, 12, replace=False):
        e = np.zeros(D)
        e[q] = h
        fd = (f(one + e, cap0)[0] - f(one - e, cap0)[0]) / (2 * h)
        errs.append(abs(fd - g_scale[q]) / max(1.0, abs(fd)))
    active = np.nonzero(g_cap)[0]
    pool = active if len(active) >= 8 else np.arange(L)
    for q in rng.choice(pool, 8, replace=False):
        e = np.zeros(L)
        e[q] = h * max(cap0[q], 1e-3)
        fd = (f(one, cap0 + e)[0] - f(one, cap0 - e)[0]) / (2 * e[q])
        errs.append(abs(fd - g_cap[q]) / max(1.0, abs(fd)))
    for _ in range(8):
        v = rng.normal(size=D)
        fd = (f(one + h * v, cap0)[0] - f(one - h * v, cap0)[0]) / (2 * h)
        errs.append(abs(fd - float(g_scale @ v)) / max(1.0, abs(fd)))
    errs = np.array(errs)
    say(f"  relative errors: median {np.median(errs):.2e}, max {errs.max():.2e}")
    say("  " + " ".join(f"{e:.1e}" for e in errs))
    # piecewise-linear map: exact up to rounding unless a clip switches inside +-h
    assert np.median(errs) <= 1e-4
    assert (errs <= 1e-3).mean() >= 0.8


def test_fp32_adjoint_on_diff_workload_close_to_fp64():
    """The differentiation workload as the benchmark runs it (FP32 iterate,
    1000 unrolled iterations, checkpoints every 50): the FP32 adjoint agrees
    with the FP64 adjoint (itself checked against the oracle and finite
    differences above) within FP32_DIFF_BAR relative for every derivative.
    The two runs take the same penalty decisions and their dispatches agree
    to about 7e-6; the derivatives differ by about 2.3e-3, the FP32
    rounding of 1000 reversed iterations (the adjoint arrays are FP32)."""
    say("[adjoint] diff workload fp32 vs fp64, 1000 iterations")
    inst = synth.config("diff")
    w = weights(inst, seed=2024)
    g64, r64, p64 = gpu_grads(inst, 1000, w, 1.0, dtype="f64", every=50)
    g32, r32, p32 = gpu_grads(inst, 1000, w, 1.0, dtype="f32", every=50)
    say(f"  penalties fp64 {r64['rho_p']:.4g}/{r64['rho_theta']:.4g}, "
        f"fp32 {r32['rho_p']:.4g}/{r32['rho_theta']:.4g}")
    say(f"  dispatch: fp32 relative error {rel(p32, p64):.2e}")
    errs = {k: rel(g32[k], g64[k]) for k in g64}
    say("  " + ", ".join(f"{k}: {v:.2e}" for k, v in errs.items()))
    assert (r32["rho_p"], r32["rho_theta"]) == (r64["rho_p"], r64["rho_theta"])
    for k, e in errs.items():
        assert e <= FP32_DIFF_BAR, (k, e)


FP32_DIFF_BAR = 5e-3


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-5), ("f32", 2e-3)])
def test_unrolled_adjoint_reaches_the_envelope_sensitivities(dtype, bar):
    """Section 5.5 on the Tiny grid: the library's adjoint of the cost after
    1500 unrolled iterations from zero equals the exact derivatives of the
    optimal cost (the node prices for the loads, minus the limit duals for
    the generator limits), computed from the exact QP independently of the
    message-passing arithmetic (tests/adj_cases.py), within `bar` relative
    to the largest derivative; after 100 iterations it does not yet."""
    from tests.adj_cases import tiny_exact_sensitivities

    say(f"[adjoint] envelope sensitivities, tiny, {dtype}")
    inst, g_load, g_pmax, _ = tiny_exact_sensitivities()
    J = len(inst.gen_node) + len(inst.load_node) + len(inst.bat_node)
    w = np.zeros((J, int(inst.T)))
    errs = []
    for n in (100, 1500):
        g, _, _ = gpu_grads(inst, n, w, 1.0, dtype=dtype, every=50)
        e_load = float((g["load"][:, 0].numpy() - g_load).__abs__().max()) / np.abs(g_load).max()
        e_pmax = float((g["pmax"][:, 0].numpy() - g_pmax).__abs__().max()) / np.abs(g_pmax).max()
        say(f"  {n} iterations: load {e_load:.2e}, pmax {e_pmax:.2e}")
        errs.append(max(e_load, e_pmax))
    assert errs[0] > bar
    assert errs[1] <= bar, errs
