"""Host-side checks of the seeded synthetic workloads: the reference
dispatch that make_instance keeps is a feasible point of the N-1 problem
with free post-outage phases (every generator within its box and ramp
limits, every line within capacity in the base case and after each
outage), checked by dense DC power flow on each post-outage network,
independently of the PTDF/LODF arithmetic that raised the capacities."""
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
