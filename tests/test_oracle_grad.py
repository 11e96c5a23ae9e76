"""The oracle's reverse-mode derivative through unrolled iterations
(Section 4.4), taken with PyTorch autograd over its FP64 steps, agrees with
central finite differences of the oracle itself.  This pins the reference
against which the library's hand-written adjoint is compared: the map is
piecewise linear, so away from a switch of some clip the central difference
is exact up to rounding."""
import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver as Oracle
from tests.adj_cases import tight, weights

N_ITERS = 60
H = 1e-6


def objective_and_dispatch(inst, load_d, cap, pmax, opts):
    o = Oracle(inst, opts, load_d=load_d, line_cap=cap, gen_pmax=pmax)
    o.run(N_ITERS)
    return o.objective(), o.dispatch()


@pytest.mark.parametrize("adapt", [0, 10])
def test_autograd_matches_central_differences(adapt):
    inst = tight()
    opts = Options(rho_p=0.3, rho_theta=2.0, eps=1e-12, adapt_every=adapt)
    w = torch.tensor(weights(inst))
    G, T = len(inst.gen_node), int(inst.T)
    base = [torch.tensor(np.asarray(inst.load_d, float)),
            torch.tensor(np.asarray(inst.line_cap, float)),
            torch.tensor(np.asarray(inst.gen_pmax, float).reshape(G, T))]
    x = [b.clone().requires_grad_(True) for b in base]
    obj, disp = objective_and_dispatch(inst, *x, opts)
    (obj + (w * disp).sum()).backward()
    grads = [xi.grad for xi in x]
    # each group has active clips (nonzero derivatives) in this run
    assert all(int((g != 0).sum()) > 0 for g in grads)

    def f(vals):
        with torch.no_grad():
            o, d = objective_and_dispatch(inst, *vals, opts)
            return float(o + (w * d).sum())

    for which, g in enumerate(grads):
        flat = g.flatten()
        picks = torch.argsort(flat.abs(), descending=True)[:3].tolist() + [0]
        for q in picks:
            idx = np.unravel_index(q, g.shape)
            up = [b.clone() for b in base]
            dn = [b.clone() for b in base]
            up[which][idx] += H
            dn[which][idx] -= H
            fd = (f(up) - f(dn)) / (2 * H)
            assert abs(float(g[idx]) - fd) <= 1e-6 * max(1.0, abs(fd)), (which, idx, float(g[idx]), fd)


def test_converged_prices_and_unrolled_derivatives_reach_the_envelope_sensitivities():
    """Section 5.5: at the optimum the derivative of the total cost with
    respect to a generator's limit is minus the limit's dual, and with
    respect to a load's demand the node's price (envelope theorem).  Both
    are computed from the exact QP (tests/adj_cases.py), independently of
    the oracle.  The converged oracle's prices -rho_p sum_k u_k equal the
    load derivatives, and its unrolled autograd derivative approaches both
    sets as the number of iterations grows (the paper's observation), to
    within 1e-5 after 1500 iterations from zero."""
    from tests.adj_cases import tiny_exact_sensitivities

    inst, g_load, g_pmax, cost = tiny_exact_sensitivities()
    assert np.abs(g_pmax).max() > 1.0  # a generator sits at its limit
    s = Oracle(inst, Options(eps=1e-9, max_iter=200000))
    r = s.solve()
    assert r.converged
    assert abs(r.objective - cost) <= 1e-6 * abs(cost)
    lmp = s.lmp()[:, 0].numpy()
    np.testing.assert_allclose(lmp[inst.load_node], g_load, rtol=1e-6)

    errs = []
    for n in (100, 1500):
        ld = torch.tensor(np.asarray(inst.load_d, float), requires_grad=True)
        pm = torch.tensor(np.asarray(inst.gen_pmax, float), requires_grad=True)
        o = Oracle(inst, Options(eps=1e-12), load_d=ld, gen_pmax=pm)
        o.run(n)
        o.objective().backward()
        e_load = np.abs(ld.grad[:, 0].numpy() - g_load).max() / np.abs(g_load).max()
        e_pmax = np.abs(pm.grad[:, 0].numpy() - g_pmax).max() / np.abs(g_pmax).max()
        errs.append(max(e_load, e_pmax))
    assert errs[1] < errs[0]
    assert errs[1] <= 1e-5, errs
