"""Instances for the derivative tests: small networks with tight line
capacities, generator limits and cheap generators, so that line, generator
and ramp clips become active within tens of iterations (otherwise the
capacity and limit derivatives of a short unrolled run are all zero)."""
import numpy as np

from paper_2410_17203_amd import synth


def tight(name="adj", N=14, L=20, G=4, D=10, B=2, T=6, K=3, seed=77):
    inst = synth.make_instance(name, N=N, L=L, G=G, D=D, B=B, T=T, K=K, seed=seed)
    inst.line_cap = np.asarray(inst.line_cap) * 0.3
    inst.gen_pmax = np.asarray(inst.gen_pmax) * 0.8
    inst.gen_c1 = np.asarray(inst.gen_c1) * 0.02
    return inst


def weights(inst, seed=0):
    """Fixed N(0, 1) weights on the device powers [G+D+B, T]."""
    J = len(inst.gen_node) + len(inst.load_node) + len(inst.bat_node)
    return np.random.default_rng(seed).normal(size=(J, int(inst.T)))


def tiny_exact_sensitivities(h=1e-6):
    """Exact derivatives of the optimal cost of the Tiny DC OPF (T = 1,
    K = 0) with respect to every load's demand and every generator's upper
    limit, independent of the message-passing arithmetic: the QP over
    generator outputs with PTDF line flows is solved exactly by active-set
    enumeration (tests/qp_enum.py); with that active set held, the optimum
    is the solution of one KKT linear system, whose central differences in
    the data give the derivatives (exact up to rounding while the active set
    is strictly complementary, which is checked: every held row moves with
    the data and no free row reaches a bound).  By the envelope theorem these
    are the prices of Section 5.5: the load derivative is the node's price
    and the capacity derivative minus the limit's dual.

    Returns (instance, d cost / d load [D], d cost / d pmax [G], cost)."""
    from tests.qp_enum import solve_qp_enum

    inst = synth.config("tiny")
    N, G = int(inst.N), len(inst.gen_node)
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    sus = np.asarray(inst.line_sus, float)
    Bm = np.zeros((N, N))
    for f, t, b in zip(frm, to, sus):
        Bm[f, f] += b
        Bm[t, t] += b
        Bm[f, t] -= b
        Bm[t, f] -= b
    X = np.zeros((N, N))
    X[1:, 1:] = np.linalg.inv(Bm[1:, 1:])
    ptdf = sus[:, None] * (X[frm] - X[to])  # line flow per unit injected at each node
    Cg = np.zeros((N, G))
    Cg[inst.gen_node, np.arange(G)] = 1.0

    def data(d, pmax):
        inj = np.zeros(N)
        np.subtract.at(inj, inst.load_node, d)
        f0 = ptdf @ inj
        C = np.vstack([np.eye(G), ptdf @ Cg])
        lo = np.r_[np.asarray(inst.gen_pmin, float)[:, 0], -np.asarray(inst.line_cap) - f0]
        hi = np.r_[pmax, np.asarray(inst.line_cap) - f0]
        return (np.diag(2 * np.asarray(inst.gen_c2)), np.asarray(inst.gen_c1, float),
                np.ones((1, G)), np.array([d.sum()]), C, lo, hi)

    d0 = np.asarray(inst.load_d, float)[:, 0].copy()
    p0 = np.asarray(inst.gen_pmax, float)[:, 0].copy()
    H, f, E, e, C, lo, hi = data(d0, p0)
    x = solve_qp_enum(H, f, E, e, C, lo, hi, max_active=G - 1)
    Cx = C @ x
    at_lo = np.abs(Cx - lo) < 1e-8
    at_hi = np.abs(Cx - hi) < 1e-8

    def solve_held(d, pmax):
        H, f, E, e, C, lo, hi = data(d, pmax)
        A = np.vstack([E, C[at_lo], C[at_hi]])
        b = np.r_[e, lo[at_lo], hi[at_hi]]
        m = A.shape[0]
        kkt = np.block([[H, A.T], [A, np.zeros((m, m))]])
        sol = np.linalg.solve(kkt, np.r_[-f, b])
        xx = sol[:G]
        return 0.5 * xx @ H @ xx + f @ xx, xx, sol[G:], (C, lo, hi)

    cost, xx, mult, (C0, lo0, hi0) = solve_held(d0, p0)
    assert np.abs(xx - x).max() <= 1e-9
    free = ~(at_lo | at_hi)
    gap = np.minimum(C0 @ xx - lo0, hi0 - C0 @ xx)[free]
    assert gap.min() > 1e3 * h, "a free row is at a bound"
    assert np.abs(mult[1:]).min() > 1e-6, "a held row has a zero multiplier"

    def fd(which, n):
        out = np.zeros(n)
        for i in range(n):
            dp = np.zeros(n)
            dp[i] = h
            args_up = (d0 + dp, p0) if which == "load" else (d0, p0 + dp)
            args_dn = (d0 - dp, p0) if which == "load" else (d0, p0 - dp)
            out[i] = (solve_held(*args_up)[0] - solve_held(*args_dn)[0]) / (2 * h)
        return out

    return inst, fd("load", len(d0)), fd("pmax", G), cost
