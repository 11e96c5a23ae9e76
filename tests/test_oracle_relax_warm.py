"""Pins of the oracle's over-relaxed iteration (Section 3.6) and of its warm
start (Section 3.4).

* At alpha = 1 the explicit-copy form is the message-passing iterate, bit
  for bit.
* For alpha = 1.5 the simplified updates of Section 3.6 (z' = alpha ptilde'
  + (1 - alpha) z, u' = u + alpha pbar', ...) equal textbook over-relaxed
  ADMM written out here with the projections onto the balance and
  consistency sets applied literally (Boyd et al., Section 3.4.3).
* The relaxed iteration reaches the exact optimum of the Tiny DC OPF and of
  the two-node dispatch.
* Exporting and re-loading the iterate continues the run bit for bit; a
  warm-started perturbed day reaches its own exact optimum.
"""
import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver, prox_generator, prox_line
from paper_2410_17203_amd import synth
from tests.test_oracle_iteration import _tiny_qp, _two_node_analytic


def _assert_same_state(a, b, exact=True, tol=0.0):
    for k in ("p", "th", "u", "v", "pbar", "thbar"):
        x, y = getattr(a, k), getattr(b, k)
        if exact:
            assert torch.equal(x, y), k
        else:
            assert float((x - y).abs().max()) <= tol * max(1.0, float(y.abs().max())), k


def test_explicit_copies_at_alpha_one_are_the_plain_iterate():
    """With alpha = 1 the copies are z = ptilde and xi = thetabar exactly, so
    the line targets and prices are the plain ones bit for bit; the device
    power target avg_k(z_k - u_k) rounds differently from p - avg_k(pbar_k +
    u_k), so the two runs agree to a few units in the last place, with the
    same penalty decisions."""
    inst = synth.config("tiny", T=4, K=3, seed=5, B=2)
    a = Solver(inst, Options(eps=1e-12))
    b = Solver(inst, Options(eps=1e-12, explicit_copies=True))
    for _ in range(40):
        ra, rb = a.step(), b.step()
        assert (ra.rho_p, ra.rho_theta) == (rb.rho_p, rb.rho_theta)
        for x, y in [(ra.primal_p, rb.primal_p), (ra.primal_th, rb.primal_th),
                     (ra.dual_p, rb.dual_p), (ra.dual_th, rb.dual_th),
                     (ra.objective, rb.objective)]:
            assert abs(x - y) <= 1e-10 * max(abs(x), 1e-300)
    _assert_same_state(a, b, exact=False, tol=1e-13)
    torch.testing.assert_close(b.z, b.p - b.pbar, rtol=0, atol=0)
    torch.testing.assert_close(b.xi, b.thbar, rtol=0, atol=0)


class _TextbookRelaxed:
    """Over-relaxed ADMM on the problem of Section 3.1 with explicit
    duplicate variables: the prox steps at z - u and xi - v, then
    p_half = alpha p + (1 - alpha) z, z = projection of p_half + u onto
    {zbar = 0} (subtract the node mean), xi = projection of theta_half + v
    onto {xitilde = 0} (the node mean), u += p_half - z, v += theta_half - xi.
    Generators and loads only, T = 1, fixed penalties."""

    def __init__(self, inst, alpha, rho_p=1.0, rho_th=1.0):
        ref = Solver(inst, Options(adapt_every=0))   # network tensors only
        self.net = net = ref.net
        self.alpha, self.rp, self.rt = alpha, rho_p, rho_th
        shape = (net.Kp, net.J, net.T)
        self.p, self.th, self.z, self.xi, self.u, self.v = [torch.zeros(shape, dtype=torch.float64)
                                                            for _ in range(6)]

    def step(self):
        net, L, G = self.net, self.net.L, self.net.G
        x, y = self.z - self.u, self.xi - self.v
        s, c = net.line_params()
        s, c = s[:, :, None], c[:, :, None]
        p1, p2, th1, th2 = prox_line(x[:, :L], x[:, L:2 * L], y[:, :L], y[:, L:2 * L],
                                     s, c, self.rp, self.rt)
        rho_hat = net.Kp * self.rp
        X, Y = x.mean(0)[2 * L:], y.mean(0)[2 * L:]
        pg = prox_generator(X[:G], rho_hat, net.gen_c2[:, None], net.gen_c1[:, None],
                            net.gen_pmin, net.gen_pmax)
        pnc = torch.cat([pg, -net.load_d], 0)
        p = torch.cat([p1, p2, pnc[None].expand(net.Kp, -1, -1)], 1)
        th = torch.cat([th1, th2, Y[None].expand(net.Kp, -1, -1)], 1)
        a = self.alpha
        ph = a * p + (1 - a) * self.z
        thh = a * th + (1 - a) * self.xi
        self.z = net.resid(ph + self.u)
        self.xi = net.avg(thh + self.v)
        self.u = self.u + ph - self.z
        self.v = self.v + thh - self.xi
        self.p, self.th = p, th


@pytest.mark.parametrize("alpha", [1.0, 1.5, 1.8])
def test_relaxed_updates_equal_textbook_overrelaxed_admm(alpha):
    inst = synth.config("tiny", K=2, seed=3)
    ora = Solver(inst, Options(alpha=alpha, explicit_copies=True, adapt_every=0, rho_p=0.7,
                               rho_theta=1.3))
    ref = _TextbookRelaxed(inst, alpha, 0.7, 1.3)
    for _ in range(60):
        ora.step()
        ref.step()
    scale = max(1.0, float(ref.u.abs().max()))
    for k in ("p", "th", "z", "xi", "u", "v"):
        got, want = getattr(ora, k), getattr(ref, k)
        assert float((got - want).abs().max()) <= 1e-11 * scale, k


def test_relaxed_iteration_reaches_the_exact_optimum():
    inst = synth.config("tiny")
    s = Solver(inst, Options(alpha=1.5, eps=1e-8, max_iter=100000))
    r = s.solve()
    assert r.converged
    x, obj = _tiny_qp(inst)
    assert abs(r.objective - obj) <= 1e-5 * abs(obj)
    np.testing.assert_allclose(s.dispatch()[:inst.G, 0].numpy(), x, atol=2e-5)
    c2, c1, pmax, d, sus = (0.5, 0.25), (1.0, 2.0), (5.0, 5.0), 3.0, 2.0
    two = synth.two_node(d=d, c2=c2, c1=c1, pmax=pmax, sus=sus, cap=1.0)
    s = Solver(two, Options(alpha=1.5, eps=1e-10, eps_relative=False, max_iter=200000))
    assert s.solve().converged
    p1, p2, _, lmp = _two_node_analytic(c2, c1, pmax, d, 1.0, sus)
    np.testing.assert_allclose(s.dispatch()[:2, 0].numpy(), [p1, p2], atol=1e-7)
    np.testing.assert_allclose(s.lmp()[:, 0].numpy(), lmp, rtol=1e-6)


@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_export_and_reload_continue_bit_for_bit(alpha):
    """A run of 100 iterations equals 60 iterations, an export, and 40 more
    iterations of a new solver loaded with that state (60 is a multiple of
    the penalty period, so the restarted count keeps the schedule)."""
    inst = synth.config("tiny", T=6, K=3, seed=8, B=2)
    opt = Options(eps=1e-12, alpha=alpha)
    a = Solver(inst, opt)
    a.run(100)
    b = Solver(inst, opt)
    b.run(60)
    c = Solver(inst, opt, init=b.export_state())
    c.run(40)
    _assert_same_state(a, c)
    assert torch.equal(a.z, c.z) and torch.equal(a.xi, c.xi)
    assert a.bat is not None and torch.equal(a.bat.lam, c.bat.lam)
    assert a.ramp is not None and torch.equal(a.ramp.lam, c.ramp.lam)
    assert (a.rho_p, a.rho_th) == (c.rho_p, c.rho_th)


def test_warm_started_next_day_reaches_its_optimum():
    """Section 3.4: the next day (loads +3%) started from the previous day's
    solution reaches the exact optimum of the next day, sooner than from
    zero."""
    day1 = synth.config("tiny")
    day2 = day1.copy()
    day2.load_d = day1.load_d * 1.03
    a = Solver(day1, Options(eps=1e-7, max_iter=100000))
    assert a.solve().converged
    warm = Solver(day2, Options(eps=1e-7, max_iter=100000), init=a.export_state())
    rw = warm.solve()
    cold = Solver(day2, Options(eps=1e-7, max_iter=100000))
    rc = cold.solve()
    assert rw.converged and rc.converged
    assert rw.iter < rc.iter
    x, obj = _tiny_qp(day2)
    assert abs(rw.objective - obj) <= 1e-5 * abs(obj)


def test_load_state_rejects_another_structure():
    a = Solver(synth.config("tiny", K=2), Options())
    a.run(3)
    with pytest.raises(ValueError):
        Solver(synth.config("tiny", K=3), Options(), init=a.export_state())
