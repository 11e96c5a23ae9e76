"""Pins of the oracle's message-passing iteration (Section 3) against things
other than itself: the Fig. 1 topology, the algebra of the average and
residual operators (Appendix B), a hand-traced first iteration, a two-node
dispatch solved analytically, the Tiny DC OPF solved exactly as a reduced
(PTDF) QP by active-set enumeration, the dual invariants, the price
identity at the fixed point, and independence from the initial penalty."""
import math
import os

import numpy as np
import pytest
import torch

from oracle.mp import Network, Options, Solver
from paper_2410_17203_amd import synth
from tests.qp_enum import solve_qp_enum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fig1_instance():
    rows, expect = [], None
    for line in open(os.path.join(GOLDEN, "fig1_network.txt")):
        line = line.strip()
        if line.startswith("#="):
            expect = [int(v) for v in line[2:].split()]
            continue
        if not line or line.startswith("#"):
            continue
        rows.append(line.split())
    f = lambda v: np.asarray(v, float)
    lines = [r for r in rows if r[1] == "line"]
    gens = [r for r in rows if r[1] == "gen"]
    loads = [r for r in rows if r[1] == "load"]
    bats = [r for r in rows if r[1] == "battery"]
    i32 = lambda v: np.asarray(v, np.int32)
    inst = synth.Instance(
        name="fig1", N=3, T=1, K=0,
        line_from=i32([int(r[2]) - 1 for r in lines]), line_to=i32([int(r[3]) - 1 for r in lines]),
        line_sus=f([1.0] * len(lines)), line_cap=f([1.0] * len(lines)), outage=i32([]),
        gen_node=i32([int(r[2]) - 1 for r in gens]), gen_c2=f([1.0] * len(gens)),
        gen_c1=f([1.0] * len(gens)), gen_pmin=np.zeros((len(gens), 1)),
        gen_pmax=np.ones((len(gens), 1)), gen_ramp=np.zeros(len(gens)),
        load_node=i32([int(r[2]) - 1 for r in loads]), load_d=np.ones((len(loads), 1)),
        bat_node=i32([int(r[2]) - 1 for r in bats]), bat_P=f([1.0] * len(bats)),
        bat_dur=f([4.0] * len(bats)), bat_eta=f([0.95] * len(bats)),
        bat_alpha=f([1.0] * len(bats)))
    return inst, expect, len(rows)


def test_fig1_topology():
    inst, (J, N, D, d1, d2, d3), ndev = _fig1_instance()
    net = Network(inst)
    assert net.J == J and net.N == N and ndev == D
    assert net.deg.tolist() == [d1, d2, d3]


def _dense_avg(net):
    """A = L' diag(|n|)^-1 L with L the node-terminal incidence (App. B)."""
    Lm = torch.zeros(net.N, net.J, dtype=torch.float64)
    Lm[net.term_node, torch.arange(net.J)] = 1.0
    return Lm.T @ torch.diag(1.0 / Lm.sum(1)) @ Lm


def test_average_operator_algebra():
    inst = synth.config("tiny")
    net = Network(inst)
    A = _dense_avg(net)
    R = torch.eye(net.J, dtype=torch.float64) - A
    torch.testing.assert_close(A @ A, A, atol=1e-14, rtol=0)
    torch.testing.assert_close(A.T, A, atol=0, rtol=0)
    torch.testing.assert_close(R @ R, R, atol=1e-14, rtol=0)
    assert float((A @ R).abs().max()) < 1e-14
    x = torch.randn(3, net.J, 2, dtype=torch.float64)
    torch.testing.assert_close(net.avg(x), torch.einsum("ij,kjt->kit", A, x), atol=1e-14, rtol=0)
    torch.testing.assert_close(net.resid(x), torch.einsum("ij,kjt->kit", R, x), atol=1e-14, rtol=0)


def test_residuals_match_dense_reexpansion():
    inst = synth.config("tiny", T=3, K=2, seed=7)
    s = Solver(inst, Options(adapt_every=0))
    net = s.net
    A = _dense_avg(net)
    R = torch.eye(net.J, dtype=torch.float64) - A
    for _ in range(12):
        p0, th0 = s.p.clone(), s.th.clone()
        r = s.step()
        dp, dth = s.p - p0, s.th - th0
        rpp = torch.linalg.norm(torch.einsum("ij,kjt->kit", A, s.p))
        rpt = torch.linalg.norm(torch.einsum("ij,kjt->kit", R, s.th))
        rdp = torch.linalg.norm(torch.einsum("ij,kjt->kit", R, dp))
        rdt = torch.linalg.norm(torch.einsum("ij,kjt->kit", A, dth))
        for a, b in [(r.primal_p, rpp), (r.primal_th, rpt), (r.dual_p, rdp), (r.dual_th, rdt)]:
            assert abs(a - float(b)) <= 1e-12 * max(1.0, float(b))


def test_hand_traced_first_iteration_and_penalty_rule():
    # Two nodes, one line (s = 1, cap = 10), G1 at node 0, G2 and a load d at
    # node 1.  From the zero start the line sees zero targets (P = 0), both
    # generators sit at pmin = 0 (c1 > 0) and the load draws d, so
    # pbar = (0, -d/3) with node degrees (2, 3); u takes that value; all
    # phases stay 0.  Hence ||pbar|| = d/sqrt(3) over the 3 terminals of
    # node 1 and ptilde = (d/3, d/3, -2d/3) there, ||dual_p|| = rho d sqrt(2/3).
    d = 6.0
    inst = synth.two_node(d=d)
    for rho0, expect_rho in [(0.01, 0.01 * 1.1), (100.0, 100.0 / 1.1), (1.0, 1.0)]:
        s = Solver(inst, Options(rho_p=rho0, adapt_every=1, eps_relative=False))
        r = s.step()
        assert math.isclose(r.primal_p, d / math.sqrt(3), rel_tol=1e-14)
        assert math.isclose(r.dual_p, rho0 * d * math.sqrt(2 / 3), rel_tol=1e-14)
        assert r.primal_th == 0.0 and r.dual_th == 0.0
        assert math.isclose(r.rms_primal, (d / math.sqrt(3)) / math.sqrt(2 * 5), rel_tol=1e-14)
        # the penalty rule of Section 3.5 with mu = 2, gamma = 1.1
        assert math.isclose(s.rho_p, expect_rho, rel_tol=1e-15)
        assert s.rho_th == 1.0
        # scaled prices are rescaled so that rho * u is unchanged
        node1 = s.net.term_node == 1
        np.testing.assert_allclose(s.rho_p * s.u[0, node1, 0].numpy(), rho0 * (-d / 3), rtol=1e-14)
        # pbar = (0, -d/3), thetas 0, P = 0
        assert float(s.p[0, 1, 0]) == 0.0
        np.testing.assert_allclose(s.pbar[0, node1, 0].numpy(), -d / 3, rtol=1e-15)


def _two_node_analytic(c2, c1, pmax, d, cap, s):
    lo = max(0.0, d - pmax[1], -cap)
    hi = min(pmax[0], cap, d)
    p1 = min(max((2 * c2[1] * d + c1[1] - c1[0]) / (2 * (c2[0] + c2[1])), lo), hi)
    p2 = d - p1
    lmp = (2 * c2[0] * p1 + c1[0], 2 * c2[1] * p2 + c1[1])
    return p1, p2, p1 / s, lmp


@pytest.mark.parametrize("cap", [10.0, 1.0])
def test_two_node_analytic_dispatch(cap):
    c2, c1, pmax, d, sus = (0.5, 0.25), (1.0, 2.0), (5.0, 5.0), 3.0, 2.0
    inst = synth.two_node(d=d, c2=c2, c1=c1, pmax=pmax, sus=sus, cap=cap)
    s = Solver(inst, Options(eps=1e-10, eps_relative=False, max_iter=200000))
    r = s.solve()
    assert r.converged
    p1, p2, dth, lmp = _two_node_analytic(c2, c1, pmax, d, cap, sus)
    pg = s.dispatch()[:2, 0].numpy()
    np.testing.assert_allclose(pg, [p1, p2], atol=1e-7)
    # flow into the to node equals p1; angle difference = flow / susceptance
    assert abs(float(s.p[0, 1, 0]) - p1) < 1e-7
    assert abs(float(s.th[0, 0, 0] - s.th[0, 1, 0]) - dth) < 1e-7
    lm = s.lmp()[:, 0].numpy()
    np.testing.assert_allclose(lm, lmp, rtol=1e-6)
    if cap == 1.0:
        assert abs(lm[1] - lm[0]) > 0.5  # congestion separates the prices


@pytest.mark.parametrize("cap", [10.0, 1.0])
def test_two_node_dc_link_dispatch(cap):
    """The same two-node economic dispatch through an HVDC link (Section 2.1):
    the dispatch, flow and prices match the closed form, and with no phase
    relation anywhere every phase stays exactly zero."""
    c2, c1, pmax, d = (0.5, 0.25), (1.0, 2.0), (5.0, 5.0), 3.0
    inst = synth.two_node(d=d, c2=c2, c1=c1, pmax=pmax, sus=2.0, cap=cap)
    inst.line_kind = np.array([1], np.int32)
    s = Solver(inst, Options(eps=1e-10, eps_relative=False, max_iter=200000))
    r = s.solve()
    assert r.converged
    p1, p2, _, lmp = _two_node_analytic(c2, c1, pmax, d, cap, 2.0)
    np.testing.assert_allclose(s.dispatch()[:2, 0].numpy(), [p1, p2], atol=1e-7)
    assert abs(float(s.p[0, 1, 0]) - p1) < 1e-7
    assert float(s.th.abs().max()) == 0.0
    np.testing.assert_allclose(s.lmp()[:, 0].numpy(), lmp, rtol=1e-6)


def test_dc_links_satisfy_optimality():
    """HVDC links in a meshed grid (T = 1, K = 0).  At the converged iterate
    (i) with the links' flows held fixed, the generator dispatch and the
    objective equal the exact QP of the remaining AC network, and (ii) each
    link's flow is optimal at the node prices: strictly inside its limit only
    where the prices at its two ends agree, at a limit only towards the higher
    price.  Together these are the optimality conditions of the full problem."""
    base = synth.config("tiny")
    inst = synth.with_dc_links(base, 3, seed=3, cap=(0.05, 0.2))
    s = Solver(inst, Options(eps=1e-9, max_iter=400000))
    r = s.solve()
    assert r.converged
    dcl = np.nonzero(inst.line_kind == 1)[0]
    f = s.canonical_state()["P"][0, dcl, 0].numpy()
    cap = inst.line_cap[dcl]
    lmp = s.lmp()[:, 0].numpy()
    # (i): the links become fixed injections (a load of f at the from node, -f at the to node)
    fixed = base.copy()
    fixed.load_node = np.r_[base.load_node, inst.line_from[dcl], inst.line_to[dcl]].astype(np.int32)
    fixed.load_d = np.r_[base.load_d, f[:, None], -f[:, None]]
    x, obj = _tiny_qp(fixed)
    assert abs(r.objective - obj) <= 1e-5 * abs(obj)
    np.testing.assert_allclose(s.dispatch()[:inst.G, 0].numpy(), x, atol=2e-5)
    # (ii)
    tol = 1e-4 * np.abs(lmp).max()
    at_limit = np.abs(f) > cap - 1e-5
    gap = lmp[inst.line_to[dcl]] - lmp[inst.line_from[dcl]]
    assert np.all(np.abs(gap[~at_limit]) <= tol)
    assert np.all(np.sign(f[at_limit]) * gap[at_limit] >= -tol)
    assert at_limit.any() and (~at_limit).any()
    assert np.abs(gap[at_limit]).max() > 1.0  # a binding link separates the prices


def _line_params_by_hand(inst):
    """Per-(k, l) susceptance and capacity written out from the instance."""
    K, L = int(inst.K), len(inst.line_from)
    sus = np.tile(np.asarray(inst.line_sus, float), (K + 1, 1))
    cap = np.tile(np.asarray(inst.line_cap, float), (K + 1, 1))
    for k in range(1, K + 1):
        o = int(inst.outage[k - 1])
        if o >= 0:
            sus[k, o] = cap[k, o] = 0.0
    if getattr(inst, "chg_k", None) is not None:
        for k, l, b, u in zip(inst.chg_k, inst.chg_line, inst.chg_sus, inst.chg_cap):
            sus[k, l], cap[k, l] = b, u
    return sus, cap


def _coupled_qp(inst):
    """The contingency-constrained problem of Section 2.3 at T = 1 as a QP in
    the generator outputs and every contingency's node phases: the lines of
    contingency k carry sus_kl (theta_f - theta_t) within cap_kl, every node
    balances in every contingency, and the generators, loads and batteries
    keep one power and one phase schedule across contingencies, so a node
    hosting any of them has the same phase in every contingency.  Solved with
    scipy's SLSQP after dropping linearly dependent equality rows."""
    from scipy.linalg import qr
    from scipy.optimize import minimize
    N, G, L, K = int(inst.N), len(inst.gen_node), len(inst.line_from), int(inst.K)
    sus, cap = _line_params_by_hand(inst)
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    dev = np.zeros(N, bool)
    dev[inst.gen_node] = dev[inst.load_node] = True
    if len(inst.bat_node):
        dev[inst.bat_node] = True
    d = np.zeros(N)
    np.add.at(d, inst.load_node, np.asarray(inst.load_d)[:, 0])
    nv = G + (K + 1) * N
    eq, rhs, ineq, bound = [], [], [], []
    for k in range(K + 1):
        F = np.zeros((L, nv))                     # flow into the to node
        F[np.arange(L), G + k * N + frm] += sus[k]
        F[np.arange(L), G + k * N + to] -= sus[k]
        B = np.zeros((N, nv))                     # net injection at each node
        B[inst.gen_node, np.arange(G)] += 1.0
        np.add.at(B, to, F)
        np.subtract.at(B, frm, F)
        eq.append(B)
        rhs.append(d)
        ineq += [F, -F]
        bound += [cap[k], cap[k]]
        if k > 0:
            for n in np.nonzero(dev)[0]:
                r = np.zeros((1, nv))
                r[0, G + k * N + n], r[0, G + n] = 1.0, -1.0
                eq.append(r)
                rhs.append(np.zeros(1))
    r = np.zeros((1, nv))
    r[0, G] = 1.0                                 # reference phase
    eq.append(r)
    rhs.append(np.zeros(1))
    A, b = np.vstack(eq), np.concatenate(rhs)
    _, R, piv = qr(A.T, pivoting=True, mode="economic")
    keep = np.sort(piv[:int((np.abs(np.diag(R)) > 1e-9 * abs(R[0, 0])).sum())])
    A, b = A[keep], b[keep]
    C, c = np.vstack(ineq), np.concatenate(bound)
    h = np.zeros(nv)
    h[:G] = 2 * np.asarray(inst.gen_c2)
    f = np.zeros(nv)
    f[:G] = inst.gen_c1
    pmin, pmax = np.asarray(inst.gen_pmin)[:, 0], np.asarray(inst.gen_pmax)[:, 0]
    x0 = np.zeros(nv)
    x0[:G] = pmax * d.sum() / pmax.sum()
    res = minimize(lambda x: 0.5 * x @ (h * x) + f @ x, x0, jac=lambda x: h * x + f,
                   method="SLSQP", bounds=[(lo, hi) for lo, hi in zip(pmin, pmax)] + [(None, None)] * (nv - G),
                   constraints=[dict(type="eq", fun=lambda x: A @ x - b, jac=lambda x: A),
                                dict(type="ineq", fun=lambda x: c - C @ x, jac=lambda x: -C)],
                   options=dict(ftol=1e-15, maxiter=3000))
    assert res.success, res.message
    return res.x[:G], float(res.fun)


def test_contingency_model_matches_phase_coupled_qp():
    """N-1 contingencies (Section 2.3) on a 14-node grid with 9 device-free
    nodes: the converged dispatch and cost equal the exact optimum of the
    contingency-constrained problem, which the contingencies make dearer
    than the base-case-only optimum."""
    inst = synth.make_instance("scopf", N=14, L=22, G=4, D=5, B=0, T=1, K=3, seed=3)
    s = Solver(inst, Options(eps=1e-9, max_iter=100000))
    r = s.solve()
    assert r.converged
    x, obj = _coupled_qp(inst)
    assert abs(r.objective - obj) <= 1e-6 * abs(obj)
    np.testing.assert_allclose(s.dispatch()[:inst.G, 0].numpy(), x, atol=1e-5)
    base = inst.copy()
    base.K, base.outage = 0, np.zeros(0, np.int32)
    assert _coupled_qp(base)[1] < obj - 1e-3 * abs(obj)


def _small_changes():
    base = synth.make_instance("chg", N=20, L=30, G=4, D=10, B=2, T=3, K=4, seed=21)
    return base, synth.with_contingency_changes(base, seed=4, second_outages=1, rating_changes=4,
                                                sus_changes=3)


def test_changed_parameters_hold_at_every_iterate():
    """General per-contingency parameters (Section 2.3): after every
    iteration each line of contingency k carries sus_kl (theta1 - theta2)
    within cap_kl, with sus_kl, cap_kl written out from the change list (a
    line taken out carries nothing)."""
    _, inst = _small_changes()
    sus, cap = _line_params_by_hand(inst)
    s = Solver(inst, Options(eps=1e-12))
    for _ in range(15):
        s.step()
        st = s.canonical_state()
        P, d = st["P"].numpy(), (st["TH1"] - st["TH2"]).numpy()
        np.testing.assert_allclose(P, sus[:, :, None] * d, rtol=0, atol=1e-12)
        assert np.all(np.abs(P) <= cap[:, :, None] + 1e-15)
    # the changed susceptances are the ones in force (not the base values)
    base_sus = np.asarray(inst.line_sus, float)
    k, l = inst.chg_k, inst.chg_line
    live = inst.chg_sus > 0
    gap = np.abs(P[k, l] - base_sus[l][:, None] * d[k, l])
    assert np.all(gap[live & (inst.chg_sus != base_sus[l])].max(1) > 1e-6)
    assert np.all(P[k[~live], l[~live]] == 0) and np.any(d[k[~live], l[~live]] != 0)


def test_change_to_zero_is_an_outage_and_base_values_change_nothing():
    """A change to (0, 0) is the N-1 outage written another way; a change to
    the base values is no change."""
    base = synth.make_instance("chg0", N=20, L=30, G=4, D=10, B=2, T=3, K=4, seed=21)
    a = Solver(base, Options(eps=1e-12))
    a.run(30)
    b_inst = base.copy()
    l = int(b_inst.outage[1])
    b_inst.outage[1] = -1
    free = [q for q in range(base.L) if q not in set(base.outage.tolist())][:3]
    b_inst.chg_k = np.array([2, 1, 3, 4], np.int32)
    b_inst.chg_line = np.array([l] + free, np.int32)
    b_inst.chg_sus = np.r_[0.0, np.asarray(base.line_sus)[free]]
    b_inst.chg_cap = np.r_[0.0, np.asarray(base.line_cap)[free]]
    b = Solver(b_inst, Options(eps=1e-12))
    b.run(30)
    sa, sb = a.canonical_state(), b.canonical_state()
    for f in sa:
        assert torch.equal(sa[f], sb[f]), f


def test_contingency_order_does_not_matter():
    """Relabelling the contingencies (outages and changes together) relabels
    the iterate and leaves the contingency means, hence the device
    schedules, unchanged up to the order of summation."""
    _, inst = _small_changes()
    perm = np.array([3, 1, 4, 2])                 # new contingency i+1 is old perm[i]
    q = inst.copy()
    q.outage = np.asarray(inst.outage)[perm - 1]
    inv = np.zeros(inst.K + 1, int)
    inv[perm] = np.arange(1, inst.K + 1)
    q.chg_k = inv[inst.chg_k].astype(np.int32)
    a, b = Solver(inst, Options(eps=1e-12)), Solver(q, Options(eps=1e-12))
    a.run(25)
    b.run(25)
    sa, sb = a.canonical_state(), b.canonical_state()
    order = np.r_[0, perm]
    for f in ["P", "TH1", "TH2", "V1", "U", "PBAR", "THBAR"]:
        torch.testing.assert_close(sb[f], sa[f][order], rtol=1e-11, atol=1e-13)
    torch.testing.assert_close(sb["PNC"], sa["PNC"], rtol=1e-11, atol=1e-13)


def _ptdf(N, frm, to, sus):
    Bm = np.zeros((N, N))
    for f, t, b in zip(frm, to, sus):
        Bm[f, f] += b
        Bm[t, t] += b
        Bm[f, t] -= b
        Bm[t, f] -= b
    X = np.zeros((N, N))
    X[1:, 1:] = np.linalg.inv(Bm[1:, 1:])
    A = np.zeros((len(frm), N))
    A[np.arange(len(frm)), frm] = 1
    A[np.arange(len(frm)), to] = -1
    return (sus[:, None] * A) @ X


def _tiny_qp(inst):
    """DC OPF (T = 1, K = 0) as a QP over generator outputs with PTDF flows."""
    N, G = inst.N, inst.G
    ptdf = _ptdf(N, inst.line_from, inst.line_to, inst.line_sus)
    Cg = np.zeros((N, G))
    Cg[inst.gen_node, np.arange(G)] = 1
    load_inj = np.zeros(N)
    np.subtract.at(load_inj, inst.load_node, inst.load_d[:, 0])
    H = np.diag(2 * inst.gen_c2)
    f = inst.gen_c1.copy()
    E = np.ones((1, G))
    e = np.array([inst.load_d[:, 0].sum()])
    Cf = ptdf @ Cg
    f0 = ptdf @ load_inj
    C = np.vstack([np.eye(G), Cf])
    lo = np.concatenate([inst.gen_pmin[:, 0], -inst.line_cap - f0])
    hi = np.concatenate([inst.gen_pmax[:, 0], inst.line_cap - f0])
    x = solve_qp_enum(H, f, E, e, C, lo, hi, max_active=G - 1)
    return x, float(0.5 * x @ H @ x + f @ x)


@pytest.fixture(scope="module")
def tiny_converged():
    inst = synth.config("tiny")
    s = Solver(inst, Options(eps=1e-8, max_iter=100000))
    r = s.solve()
    return inst, s, r


def test_tiny_matches_exact_qp(tiny_converged):
    inst, s, r = tiny_converged
    assert r.converged
    x, obj = _tiny_qp(inst)
    assert abs(r.objective - obj) <= 1e-5 * abs(obj)
    np.testing.assert_allclose(s.dispatch()[:inst.G, 0].numpy(), x, atol=2e-5)


def test_tiny_price_identity(tiny_converged):
    # At a fixed point of step 2 with pbar = 0 an interior generator satisfies
    # 2 c2 p + c1 + (K+1) rho_p avg_k u_k = 0, i.e. its marginal cost equals
    # the locational price -rho_p sum_k u_k.
    inst, s, r = tiny_converged
    pg = s.dispatch()[:inst.G, 0].numpy()
    lmp = s.lmp()[:, 0].numpy()
    interior = (pg > 1e-4) & (pg < inst.gen_pmax[:, 0] - 1e-4)
    assert interior.any()
    mc = 2 * inst.gen_c2 * pg + inst.gen_c1
    np.testing.assert_allclose(mc[interior], lmp[inst.gen_node[interior]], rtol=1e-5)


def test_dual_invariants_hold_along_iterations():
    inst = synth.config("tiny", T=4, K=3, seed=5, B=2)
    s = Solver(inst, Options())
    for _ in range(40):
        s.step()
        # u constant within every node (u tilde = 0), v sums to zero per node
        assert float(s.net.resid(s.u).abs().max()) <= 1e-13 * max(1.0, float(s.u.abs().max()))
        vs = s.net.node_sum(s.v)
        assert float(vs.abs().max()) <= 1e-12 * max(1.0, float(s.v.abs().sum()))


def test_noop_contingencies_reach_base_solution():
    base = synth.config("tiny")
    a = Solver(base, Options(eps=1e-8, max_iter=100000))
    ra = a.solve()
    cont = base.copy()
    cont.K = 2
    cont.outage = np.array([-1, -1], np.int32)
    b = Solver(cont, Options(eps=1e-8, max_iter=100000))
    rb = b.solve()
    assert ra.converged and rb.converged
    np.testing.assert_allclose(b.dispatch().numpy(), a.dispatch().numpy(), atol=1e-5)
    assert abs(ra.objective - rb.objective) <= 1e-6 * abs(ra.objective)


def test_solution_independent_of_initial_penalty(tiny_converged):
    inst, s, r = tiny_converged
    b = Solver(inst, Options(eps=1e-8, max_iter=100000, rho_p=4.0, rho_theta=0.3))
    rb = b.solve()
    assert rb.converged
    np.testing.assert_allclose(b.dispatch().numpy(), s.dispatch().numpy(), atol=2e-5)
    np.testing.assert_allclose(b.lmp().numpy(), s.lmp().numpy(), rtol=1e-4)


def test_curtailable_load_sets_the_price():
    """Section 2.1: a curtailable load is a generator with pmin = -d < pmax = 0
    and linear cost.  With demand above the total generator capacity and an
    uncongested line, both generators run at capacity, the load is served
    with exactly that power, and the price at both nodes is the curtailment
    cost (the marginal value of the unserved demand)."""
    cost, d = 50.0, 3.0
    base = synth.two_node(d=d, c2=(0.5, 0.25), c1=(1.0, 2.0), pmax=(1.0, 0.5), cap=10.0)
    inst = synth.with_curtailable_loads(base, cost=cost)
    s = Solver(inst, Options(eps=1e-9, eps_relative=False, max_iter=400000))
    r = s.solve()
    assert r.converged
    p = s.dispatch()[:, 0].numpy()
    np.testing.assert_allclose(p, [1.0, 0.5, -1.5], atol=1e-6)
    np.testing.assert_allclose(s.lmp()[:, 0].numpy(), [cost, cost], rtol=1e-5)


def _battery_grid():
    """Two nodes, one line, two periods: a cheap generator at node 0, a dear
    one, a load and a battery (charge efficiency 0.9, discharge cost 1) at
    node 1.  The load peaks in the second period, when the line is
    congested, so the battery charges in the first and discharges in the
    second."""
    f = lambda v: np.asarray(v, dtype=np.float64)
    return synth.Instance(
        name="battery2", N=2, T=2, K=0,
        line_from=np.array([0], np.int32), line_to=np.array([1], np.int32),
        line_sus=f([4.0]), line_cap=f([1.8]), outage=np.zeros(0, np.int32),
        gen_node=np.array([0, 1], np.int32), gen_c2=f([0.05, 0.5]), gen_c1=f([10.0, 30.0]),
        gen_pmin=np.zeros((2, 2)), gen_pmax=f([[4.0, 4.0], [5.0, 5.0]]), gen_ramp=np.zeros(2),
        load_node=np.array([1], np.int32), load_d=f([[1.0, 3.0]]),
        bat_node=np.array([1], np.int32), bat_P=f([0.6]), bat_dur=f([2.0]), bat_eta=f([0.9]),
        bat_alpha=f([1.0]), meta={})


def _battery_qp(inst):
    """The two-node, two-period problem as an exact QP over x = (g0_1, g0_2,
    g1_1, g1_2, c_1, c_2, delta_1, delta_2): generator cost plus the
    battery's discharge cost alpha (delta_1 + delta_2) (Section 2.1),
    balance at node 1 in each period (the line carries g0_t), the state of
    charge s_2 = eta c_1 - delta_1 within [0, dur P] and back to zero at the
    end, every box, and the line capacity folded into g0's bounds."""
    c2, c1 = np.asarray(inst.gen_c2), np.asarray(inst.gen_c1)
    eta, alpha = float(inst.bat_eta[0]), float(inst.bat_alpha[0])
    P, smax = float(inst.bat_P[0]), float(inst.bat_dur[0] * inst.bat_P[0])
    cap, d = float(inst.line_cap[0]), np.asarray(inst.load_d)[0]
    H = np.diag([2 * c2[0], 2 * c2[0], 2 * c2[1], 2 * c2[1], 0, 0, 0, 0])
    f = np.array([c1[0], c1[0], c1[1], c1[1], 0, 0, alpha, alpha])
    E = np.array([[1, 0, 1, 0, -1, 0, 1, 0],
                  [0, 1, 0, 1, 0, -1, 0, 1],
                  [0, 0, 0, 0, eta, eta, -1, -1]], float)
    e = np.array([d[0], d[1], 0.0])
    C = np.vstack([np.eye(8), [[0, 0, 0, 0, eta, 0, -1, 0]]])
    pm = np.asarray(inst.gen_pmax)
    lo = np.array([0, 0, 0, 0, 0, 0, 0, 0, 0], float)
    hi = np.array([min(pm[0, 0], cap), min(pm[0, 1], cap), pm[1, 0], pm[1, 1], P, P, P, P, smax])
    x = solve_qp_enum(H, f, E, e, C, lo, hi)
    return x, float(0.5 * x @ H @ x + f @ x)


def test_battery_dispatch_and_cost_match_exact_qp():
    """A converged solve with a battery in use: the dispatch, the battery's
    charge and discharge and the objective, which includes alpha * sum(delta),
    equal the exact QP.  Costing the charge instead of the discharge, or
    reading the wrong slice of the battery state, moves the objective by
    more than the tolerance."""
    inst = _battery_grid()
    x, obj = _battery_qp(inst)
    c, dl = x[4:6], x[6:8]
    assert dl[1] > 0.1 and c[0] > 0.1          # the battery cycles
    assert abs(float(inst.bat_alpha[0]) * (dl.sum() - c.sum())) > 1e-3 * abs(obj)
    s = Solver(inst, Options(eps=1e-10, eps_relative=False, max_iter=400000))
    r = s.solve()
    assert r.converged
    assert abs(r.objective - obj) <= 1e-6 * abs(obj)
    np.testing.assert_allclose(s.dispatch()[:2].numpy().ravel(), x[:4], atol=1e-6)
    np.testing.assert_allclose(s.dispatch()[3].numpy(), dl - c, atol=1e-6)
    np.testing.assert_allclose(s.bat.delta[0].numpy(), dl, atol=1e-6)
