"""Host-side checks of the seeded synthetic workloads: the reference
dispatch that make_instance keeps is a feasible point of the N-1 problem
with free post-outage phases (every generator within its box and ramp
limits, every line within capacity in the base case and after each
outage), checked by dense DC power flow on each post-outage network,
independently of the PTDF/LODF arithmetic that raised the capacities, and
of the problem of Section 2.3 as posed (device phases shared by all
contingencies): the outaged lines carry no power, so the base phases serve
every contingency."""
import numpy as np
import pytest

from paper_2410_17203_amd import synth


def _dense_flows(N, frm, to, sus, inj):
    """DC power flow by a dense solve of the reduced susceptance Laplacian."""
    B = np.zeros((N, N))
    for f, t, b in zip(frm, to, sus):
        B[f, f] += b
        B[t, t] += b
        B[f, t] -= b
        B[t, f] -= b
    th = np.zeros((N, inj.shape[1]))
    th[1:] = np.linalg.solve(B[1:, 1:], inj[1:])
    return sus[:, None] * (th[frm] - th[to]), th


@pytest.mark.parametrize("name,over", [("tiny", dict(K=3)), ("tiny", dict(T=24, K=5, seed=9)),
                                       ("medium", dict(K=12))])
def test_reference_dispatch_is_n1_feasible(name, over):
    inst = synth.config(name, **over)
    N, T, K = int(inst.N), int(inst.T), int(inst.K)
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    sus, cap = np.asarray(inst.line_sus, float), np.asarray(inst.line_cap, float)
    disp = np.asarray(inst.meta["ref_dispatch"])
    assert np.all(disp >= np.asarray(inst.gen_pmin) - 1e-12)
    assert np.all(disp <= np.asarray(inst.gen_pmax) + 1e-12)
    if T > 1:
        assert np.all(np.abs(np.diff(disp, axis=1)) <= np.asarray(inst.gen_ramp)[:, None] + 1e-12)
    inj = np.zeros((N, T))
    np.add.at(inj, inst.gen_node, disp)
    np.subtract.at(inj, inst.load_node, np.asarray(inst.load_d))
    assert np.abs(inj.sum(0)).max() < 1e-9
    for k in range(K + 1):
        keep = np.ones(len(frm), bool)
        if k > 0:
            keep[inst.outage[k - 1]] = False
        f, th = _dense_flows(N, frm[keep], to[keep], sus[keep], inj)
        # Kirchhoff's current law holds at every node
        net = np.zeros((N, T))
        np.add.at(net, to[keep], f)
        np.subtract.at(net, frm[keep], f)
        assert np.abs(inj + net).max() < 1e-9
        assert np.all(np.abs(f) <= cap[keep][:, None] * (1 + 1e-12)), f"contingency {k} overloads"


@pytest.mark.parametrize("name,over", [("tiny", dict(K=3)), ("tiny", dict(T=24, K=3, seed=9)),
                                       ("medium", dict(K=12)), ("diff", dict())])
def test_reference_dispatch_is_feasible_with_shared_device_phases(name, over):
    """Section 2.3 as posed: one power and one phase schedule per device
    node for all contingencies.  The reference dispatch's base phases (dense
    solve), used unchanged in every contingency, must satisfy each
    contingency's balance without its outaged line and every capacity,
    which holds because the outaged lines carry no power."""
    inst = synth.config(name, **over)
    N, T, K = int(inst.N), int(inst.T), int(inst.K)
    assert K == inst.meta["K_idle"] == over.get("K", synth.CONFIGS[name]["K"])
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    sus, cap = np.asarray(inst.line_sus, float), np.asarray(inst.line_cap, float)
    disp = np.asarray(inst.meta["ref_dispatch"])
    assert np.all(disp >= np.asarray(inst.gen_pmin) - 1e-12)
    assert np.all(disp <= np.asarray(inst.gen_pmax) + 1e-12)
    if T > 1:
        assert np.all(np.abs(np.diff(disp, axis=1)) <= np.asarray(inst.gen_ramp)[:, None] + 1e-12)
    inj = np.zeros((N, T))
    np.add.at(inj, inst.gen_node, disp)
    np.subtract.at(inj, inst.load_node, np.asarray(inst.load_d))
    _, th = _dense_flows(N, frm, to, sus, inj)
    flow = sus[:, None] * (th[frm] - th[to])
    scale = np.abs(flow).max()
    assert np.abs(flow[inst.outage]).max() <= 1e-9 * scale, "an outaged line carries power"
    for k in range(K + 1):
        keep = np.ones(len(frm), bool)
        if k > 0:
            keep[inst.outage[k - 1]] = False
        net = np.zeros((N, T))
        np.add.at(net, to[keep], flow[keep])
        np.subtract.at(net, frm[keep], flow[keep])
        assert np.abs(inj + net).max() <= 1e-9 * max(1.0, scale), f"contingency {k} unbalanced"
        assert np.all(np.abs(flow[keep]) <= cap[keep][:, None] * (1 + 1e-12))


def test_uniform_outages_are_generally_infeasible_with_shared_device_phases():
    """Why the outages are chosen as they are: with uniformly drawn outages on
    a grid where most nodes host a device, no generator redispatch idles
    every outaged line (the flows of some outaged lines do not depend on the
    generators independently of the others: the constraint rows have lower
    rank than the number of outages plus the balance)."""
    inst = synth.config("medium", outage_rule="uniform")
    N, T = int(inst.N), int(inst.T)
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    sus = np.asarray(inst.line_sus, float)
    B = np.zeros((N, N))
    for f, t, b in zip(frm, to, sus):
        B[f, f] += b
        B[t, t] += b
        B[f, t] -= b
        B[t, f] -= b
    X = np.zeros((N, N))
    X[1:, 1:] = np.linalg.inv(B[1:, 1:])
    out = np.asarray(inst.outage)
    S = sus[out][:, None] * (X[frm[out]] - X[to[out]])  # outaged flow per unit injection
    A = np.vstack([np.ones(len(inst.gen_node)), S[:, inst.gen_node]])
    assert np.linalg.matrix_rank(A) < A.shape[0]


def test_batch_instances_are_all_feasible_with_shared_device_phases():
    """Every instance of the uneven batch keeps only idle outages."""
    for inst in synth.batched():
        assert inst.meta["K_idle"] == inst.K <= inst.meta["K_requested"]
        disp = np.asarray(inst.meta["ref_dispatch"])
        assert np.all(disp <= np.asarray(inst.gen_pmax) + 1e-12)
        assert np.all(disp >= 0)
