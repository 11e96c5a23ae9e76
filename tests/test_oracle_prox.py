"""Pins of the oracle's proximal operators against brute force and exact QPs.

* generator and line prox (Section 4.2) against golden-section minimisers
  that know nothing of the closed forms;
* ramp-generator and battery prox (Section 2.1 device costs, evaluated by
  the inner ADMM of Appendix D) against the exact prox from active-set
  enumeration, with enough inner iterations to converge.
"""
import numpy as np
import pytest
import torch

from oracle.mp import BatteryProx, RampProx, prox_generator, prox_line
from tests.qp_enum import solve_qp_enum

GR = (np.sqrt(5.0) - 1.0) / 2.0


def golden_min(fun, a, b, iters=100):
    """Vectorised golden-section minimiser of convex 1-D functions on [a, b]."""
    a = np.array(a, float)
    b = np.array(b, float)
    for _ in range(iters):
        c = b - GR * (b - a)
        d = a + GR * (b - a)
        left = fun(c) <= fun(d)
        b = np.where(left, d, b)
        a = np.where(left, a, c)
    return 0.5 * (a + b)


def test_generator_prox_bruteforce():
    rng = np.random.default_rng(1)
    n = 4000
    x = rng.uniform(-5, 5, n)
    rho = rng.uniform(0.1, 50, n)
    c2 = rng.uniform(0.01, 0.1, n)
    c2[: n // 3] = 0.0  # linear cost (curtailable loads, Section 2.1)
    c1 = rng.uniform(10, 50, n) * rng.choice([-1, 1], n) / 10
    pmin = rng.uniform(-2, 0.5, n)
    pmax = pmin + rng.uniform(0.0, 3, n)
    f = lambda p: c2 * p * p + c1 * p + 0.5 * rho * (p - x) ** 2
    ref = golden_min(f, pmin, pmax)
    got = prox_generator(torch.tensor(x), torch.tensor(rho), torch.tensor(c2),
                         torch.tensor(c1), torch.tensor(pmin), torch.tensor(pmax)).numpy()
    assert np.all(got >= pmin) and np.all(got <= pmax)
    np.testing.assert_allclose(got, ref, atol=2e-7)
    # both regimes are exercised
    clipped = (np.abs(got - pmin) < 1e-12) | (np.abs(got - pmax) < 1e-12)
    assert 0.1 < clipped.mean() < 0.9


def _line_bruteforce(z1, z2, xi1, xi2, s, c, rp, rt):
    """min over (P, th1, th2) of the line prox objective by nested golden
    section: outer over the flow P in [-c, c], inner over th2 with
    th1 = th2 + P/s (the susceptance equality)."""
    span = np.abs(xi1) + np.abs(xi2) + 4 * c / s + 1.0

    def inner(P):
        g = lambda t2: 0.5 * rt * ((t2 + P / s - xi1) ** 2 + (t2 - xi2) ** 2)
        t2 = golden_min(g, -span, span)
        return t2, g(t2)

    def outer(P):
        _, gv = inner(P)
        return 0.5 * rp * ((-P - z1) ** 2 + (P - z2) ** 2) + gv

    P = golden_min(outer, -c, c)
    t2, _ = inner(P)
    return P, t2 + P / s, t2


def test_line_prox_bruteforce():
    rng = np.random.default_rng(2)
    n = 1500
    z1, z2 = rng.normal(0, 2, n), rng.normal(0, 2, n)
    xi1, xi2 = rng.normal(0, 0.5, n), rng.normal(0, 0.5, n)
    s = rng.uniform(0.5, 20, n)
    c = rng.uniform(0.05, 3, n)
    rp, rt = rng.uniform(0.1, 10, n), rng.uniform(0.1, 10, n)
    P, t1, t2 = _line_bruteforce(z1, z2, xi1, xi2, s, c, rp, rt)
    T = lambda a: torch.tensor(a)
    p1, p2, th1, th2 = [v.numpy() for v in prox_line(T(z1), T(z2), T(xi1), T(xi2), T(s), T(c), T(rp), T(rt))]
    np.testing.assert_allclose(p2, P, atol=2e-6)
    np.testing.assert_allclose(p1, -P, atol=2e-6)
    np.testing.assert_allclose(th1, t1, atol=2e-6)
    np.testing.assert_allclose(th2, t2, atol=2e-6)
    # susceptance relation holds to rounding at every output
    np.testing.assert_allclose(p2, s * (th1 - th2), atol=1e-12)
    clipped = np.abs(np.abs(p2) - c) < 1e-12
    assert 0.1 < clipped.mean() < 0.9


def test_line_prox_worked_example():
    # rho = 1, s = 1, z = 0, xi = (1, 0): the 1-D problem
    # min 1/2 (2 P^2) + 1/4 (P - 1)^2 has P = 1/5 (the printed denominator of
    # Section 4.2 would give 1/9).
    one = torch.tensor(1.0, dtype=torch.float64)
    zero = torch.tensor(0.0, dtype=torch.float64)
    ten = torch.tensor(10.0, dtype=torch.float64)
    p1, p2, th1, th2 = prox_line(zero, zero, one, zero, one, ten, one, one)
    assert abs(float(p2) - 0.2) < 1e-15
    assert abs(float(th1) - 0.6) < 1e-15 and abs(float(th2) - 0.4) < 1e-15


def test_line_prox_outage_and_zero_capacity():
    rng = np.random.default_rng(3)
    n = 64
    z1, z2, xi1, xi2 = [torch.tensor(rng.normal(0, 1, n)) for _ in range(4)]
    zero = torch.zeros(n)
    p1, p2, th1, th2 = prox_line(z1, z2, xi1, xi2, zero.double(), zero.double(), 1.0, 1.0)
    assert torch.all(p2 == 0) and torch.all(p1 == 0)
    assert torch.equal(th1, xi1) and torch.equal(th2, xi2)
    # live line with zero capacity: no flow, both phases at the mean
    s = torch.full((n,), 7.0, dtype=torch.float64)
    p1, p2, th1, th2 = prox_line(z1, z2, xi1, xi2, s, zero.double(), 1.0, 2.0)
    assert torch.all(p2 == 0)
    torch.testing.assert_close(th1, 0.5 * (xi1 + xi2), rtol=0, atol=1e-15)
    torch.testing.assert_close(th2, 0.5 * (xi1 + xi2), rtol=0, atol=1e-15)


def test_dc_link_prox_brute_force():
    """HVDC link (Section 2.1): the prox of I{p1 + p2 = 0} + I{|p2| <= c} with
    no phase relation, against golden-section minimisation of the 1-D
    objective rho_p/2 ((-P - z1)^2 + (P - z2)^2) over [-c, c]; the phases
    keep their targets whatever the susceptance."""
    rng = np.random.default_rng(11)
    n = 1000
    z1, z2 = rng.normal(0, 2, n), rng.normal(0, 2, n)
    xi1, xi2 = rng.normal(0, 0.5, n), rng.normal(0, 0.5, n)
    s = rng.uniform(0.5, 20, n)
    c = rng.uniform(0.05, 3, n)
    rp, rt = rng.uniform(0.1, 10, n), rng.uniform(0.1, 10, n)
    P = golden_min(lambda x: 0.5 * rp * ((-x - z1) ** 2 + (x - z2) ** 2), -c, c)
    T = lambda a: torch.tensor(a)
    dc = torch.ones(n, dtype=torch.bool)
    p1, p2, th1, th2 = [v.numpy() for v in prox_line(T(z1), T(z2), T(xi1), T(xi2), T(s), T(c),
                                                     T(rp), T(rt), dc)]
    np.testing.assert_allclose(p2, P, atol=2e-6)
    assert np.array_equal(p1, -p2)
    assert np.array_equal(th1, xi1) and np.array_equal(th2, xi2)
    clipped = np.abs(np.abs(p2) - c) < 1e-12
    assert 0.1 < clipped.mean() < 0.9
    # the susceptance plays no part; an outaged link (c = 0) carries nothing
    q = prox_line(T(z1), T(z2), T(xi1), T(xi2), T(2 * s + 1), T(c), T(rp), T(rt), dc)
    assert np.array_equal(q[1].numpy(), p2)
    q = prox_line(T(z1), T(z2), T(xi1), T(xi2), T(0 * s), T(0 * c), T(rp), T(rt), dc)
    assert np.all(q[1].numpy() == 0) and np.array_equal(q[2].numpy(), xi1)
    # mixed masks select per element
    mix = torch.tensor(rng.random(n) < 0.5)
    m = prox_line(T(z1), T(z2), T(xi1), T(xi2), T(s), T(c), T(rp), T(rt), mix)
    ac = prox_line(T(z1), T(z2), T(xi1), T(xi2), T(s), T(c), T(rp), T(rt))
    for a, b, d in zip(m, ac, (p1, p2, th1, th2)):
        an = a.numpy()
        assert np.array_equal(an[mix.numpy()], d[mix.numpy()])
        assert np.array_equal(an[~mix.numpy()], b.numpy()[~mix.numpy()])


# ---- time-coupled devices ------------------------------------------------

def _ramp_exact(c2, c1, pmin, pmax, R, rho_hat, X):
    T = X.shape[0]
    H = (2 * c2 + rho_hat) * np.eye(T)
    f = c1 * np.ones(T) - rho_hat * X
    Dm = np.zeros((T - 1, T))
    for t in range(T - 1):
        Dm[t, t], Dm[t, t + 1] = -1, 1
    C = np.vstack([np.eye(T), Dm])
    lo = np.concatenate([pmin, -R * np.ones(T - 1)])
    hi = np.concatenate([pmax, R * np.ones(T - 1)])
    return solve_qp_enum(H, f, None, None, C, lo, hi)


@pytest.mark.parametrize("T", [2, 3])
def test_ramp_prox_converges_to_exact(T):
    rng = np.random.default_rng(10 + T)
    n = 12
    c2 = rng.uniform(0.01, 0.1, n)
    c1 = rng.uniform(10, 50, n)
    pmax = rng.uniform(1, 3, (n, T))
    pmin = np.zeros((n, T))
    R = 0.3 * pmax[:, 0]
    rho_hat = 30.0
    X = rng.uniform(-1, 4, (n, T))
    prox = RampProx(torch.tensor(c2), torch.tensor(c1), torch.tensor(pmin),
                    torch.tensor(pmax), torch.tensor(R), T)
    got = prox(torch.tensor(X), rho_hat, rho_hat, 6000).numpy()
    ref = np.stack([_ramp_exact(c2[i], c1[i], pmin[i], pmax[i], R[i], rho_hat, X[i])
                    for i in range(n)])
    np.testing.assert_allclose(got, ref, atol=1e-8)
    # at least one case with an active ramp limit
    assert np.any(np.abs(np.abs(np.diff(ref, axis=1)) - R[:, None]) < 1e-9)


def _battery_exact(P, dur, eta, alpha, rho_hat, X):
    """Exact battery prox in (c, delta) space with the state of charge
    s_{t+1} = sum_{tau<=t} (eta c_tau - delta_tau) eliminated."""
    T = X.shape[0]
    I = np.eye(T)
    H = rho_hat * np.block([[I, -I], [-I, I]])
    f = np.concatenate([rho_hat * X, alpha - rho_hat * X])
    cum = np.tril(np.ones((T, T)))
    S = np.hstack([eta * cum, -cum])           # rows: s_2 .. s_{T+1}
    E = S[T - 1:T]                             # s_{T+1} = 0
    C = np.vstack([np.eye(2 * T), S[:T - 1]])
    lo = np.zeros(2 * T + T - 1)
    hi = np.concatenate([P * np.ones(2 * T), dur * P * np.ones(T - 1)])
    x = solve_qp_enum(H, f, E, np.zeros(1), C, lo, hi)
    return x[:T], x[T:]


@pytest.mark.parametrize("T", [1, 2, 3])
def test_battery_prox_converges_to_exact(T):
    rng = np.random.default_rng(20 + T)
    n = 10
    P = rng.uniform(0.25, 1.0, n)
    dur = np.full(n, 4.0)
    eta = np.full(n, 0.95)
    alpha = np.full(n, 1.0)
    rho_hat = 5.0
    X = rng.uniform(-1.5, 1.5, (n, T)) * P[:, None]
    prox = BatteryProx(torch.tensor(P), torch.tensor(dur), torch.tensor(eta),
                       torch.tensor(alpha), T)
    got = prox(torch.tensor(X), rho_hat, rho_hat, 8000).numpy()
    exact = [_battery_exact(P[i], dur[i], eta[i], alpha[i], rho_hat, X[i]) for i in range(n)]
    c_ref = np.stack([e[0] for e in exact])
    d_ref = np.stack([e[1] for e in exact])
    np.testing.assert_allclose(got, d_ref - c_ref, atol=1e-8)
    # the discharge itself (the objective costs alpha * sum(delta), Section
    # 2.1): with alpha > 0 and eta < 1 the split of p into delta - c is
    # unique, so the oracle's delta must be the exact one, not merely its
    # difference with c
    np.testing.assert_allclose(prox.delta.numpy(), d_ref, atol=1e-8)
    if T > 1:
        assert np.any(d_ref > 1e-3) and np.any(c_ref > 1e-3)
    if T == 1:
        # a one-step battery can only dissipate: p = delta - c <= 0
        assert np.all(got <= 1e-9)
