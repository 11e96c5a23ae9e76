"""FP64 CPU oracle of proximal message passing for contingency-constrained
DC OPF (Degleris, El Gamal, Rajagopal, "GPU Accelerated Security Constrained
Optimal Power Flow", arXiv 2410.17203).

TEST INFRASTRUCTURE ONLY.  This module is imported by the test-suite, by the
smoke check and by the CPU-baseline leg of the benchmark, and by nothing
else.  It shares no code with the HIP library: it is a plain, slow,
obviously-correct restatement of the paper's iteration in float64 PyTorch CPU
ops (which also gives reverse- and forward-mode gradients for free).

Variables follow the paper's notation and layout (Section 4.1): every
terminal of every contingency carries a power p, a phase theta and scaled
duals u, v, stored as (K+1) x J x T tensors.  The non-contingency devices'
schedules are shared by all contingencies (Section 2.3) and are broadcast
along the first axis.

Terminal order: terminal 1 of every line, terminal 2 of every line, then
generators, fixed loads, batteries.  Line terminal 1 sits at the line's from
node and terminal 2 at its to node.

Readings of the paper used here (each also listed in the design notes):
  * generator prox: the first-order condition of the generator cost plus
    the proximal term gives (rho x - b) / (2a + rho) before projection; the
    printed fraction in Section 4.2 is inverted;
  * line prox: eliminating the mean phase leaves a 1-D quadratic in p2 whose
    curvature is 2 rho_p + rho_theta / (2 b^2) and whose linear term is
    rho_p (z2 - z1) + rho_theta (xi1 - xi2) / (2 b); the printed denominator
    in Section 4.2 is garbled;
  * an outaged line (b = 0) carries no power and leaves both phases free;
  * the non-contingency target is p - avg_k(pbar_k + u_k): avg_k(z_k - u_k)
    with z_k = ptilde_k (Section 3.2), the printed sign is a typo;
  * residual norms run over terminal copies (node values repeat |n| times),
    the dual phase residual uses thetabar of contingency k (the printed
    index K is a typo);
  * the penalty adapts after iterations adapt_every, 2 adapt_every, ...
    using that iteration's residuals; the scaled duals are rescaled by
    rho_old / rho_new (Section 3.5);
  * a ramp-limited generator is a generator plus |p_{t+1} - p_t| <= R;
  * time-coupled devices (ramp generator, battery) evaluate their prox with
    a fixed number of inner ADMM iterations (Appendix D) in which the
    device equalities stay in the x-update, the bounds are split off with
    copies beta and scaled duals lambda of penalty omega = scale * rho_hat,
    (beta, lambda) start at zero and are carried across outer iterations,
    lambda is rescaled with omega, and the x-iterate of the last inner
    iteration is returned;
  * an HVDC link (Section 2.1 names it without a cost) is lossless power
    transfer within its capacity with no phase relation: its prox takes the
    clipped midpoint (z2 - z1)/2 as the flow and leaves both phases at their
    targets;
  * general contingency parameters (Section 2.3): a listed (k, line) pair
    overrides the base susceptance and capacity in contingency k; a zero
    susceptance takes an AC line out, and a DC link uses only the capacity;
  * a curtailable load is a generator with pmin = -d < pmax = 0 and a
    linear cost (c2 = 0);
  * over-relaxation (Section 3.6) keeps the duplicate variables z (per
    terminal copy) and xi (node-constant) as state: the prox targets are
    z - u and xi - v, z' = alpha ptilde' + (1 - alpha) z,
    xi' = alpha thetabar' + (1 - alpha) xi, u' = u + alpha pbar',
    v' = v + alpha thetatilde'; the dual residuals are rho ||z' - z|| and
    rho ||xi' - xi|| (the plain ones when alpha = 1, where z = ptilde and
    xi = thetabar);
  * a warm start (Section 3.4) replaces the whole iterate, the inner ADMM
    state of the time-coupled devices and the penalties with those of
    another run on a network of the same structure, and restarts the
    iteration count (and so the adaptive-penalty schedule) at zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

DT = torch.float64


@dataclass
class Options:
    rho_p: float = 1.0
    rho_theta: float = 1.0
    mu: float = 2.0
    gamma: float = 1.1
    adapt_every: int = 10          # 0 disables the adaptive penalty
    eps: float = 1e-3
    eps_relative: bool = True      # tolerance scaled by the RMS load
    max_iter: int = 10000
    min_iter: int = 0
    inner_iters: int = 10
    inner_omega_scale: float = 1.0
    # over-relaxation (Section 3.6): alpha in [1, 2); explicit_copies keeps the
    # duplicate variables (z, xi) as state even at alpha = 1
    alpha: float = 1.0
    explicit_copies: bool = False


def _t(x, dtype=DT):
    if isinstance(x, torch.Tensor):
        return x.to(dtype)
    return torch.as_tensor(x, dtype=dtype)


class Network:
    """Problem data as CPU tensors, in terminal order (see module doc)."""

    def __init__(self, inst, load_d=None, line_cap=None, gen_pmax=None):
        self.N, self.T, self.K = int(inst.N), int(inst.T), int(inst.K)
        self.Kp = self.K + 1
        self.L = int(len(inst.line_from))
        self.G = int(len(inst.gen_node))
        self.D = int(len(inst.load_node))
        self.B = int(len(inst.bat_node))
        self.Jnc = self.G + self.D + self.B
        self.J = 2 * self.L + self.Jnc
        lf = torch.as_tensor(inst.line_from, dtype=torch.long)
        lt = torch.as_tensor(inst.line_to, dtype=torch.long)
        self.line_from, self.line_to = lf, lt
        self.term_node = torch.cat([lf, lt,
                                    torch.as_tensor(inst.gen_node, dtype=torch.long),
                                    torch.as_tensor(inst.load_node, dtype=torch.long),
                                    torch.as_tensor(inst.bat_node, dtype=torch.long)])
        self.deg = torch.zeros(self.N, dtype=DT).index_add_(
            0, self.term_node, torch.ones(self.J, dtype=DT))
        self.sus = _t(inst.line_sus)
        kind = getattr(inst, "line_kind", None)
        self.dc = (torch.zeros(self.L, dtype=torch.bool) if kind is None
                   else torch.as_tensor(np.asarray(kind) == 1))
        self.cap = _t(inst.line_cap) if line_cap is None else line_cap
        outage = torch.as_tensor(inst.outage, dtype=torch.long)
        # contingency k (0 = base case) keeps line l iff l != outage[k-1]
        alive = torch.ones(self.Kp, self.L, dtype=DT)
        for k in range(1, self.Kp):
            o = int(outage[k - 1])
            if o >= 0:
                alive[k, o] = 0.0
        self.alive = alive
        # general contingency parameters (Section 2.3: contingency k may set
        # any line's parameters x_kl); an entry overrides the base values
        ck = getattr(inst, "chg_k", None)
        self.chg = torch.zeros(self.Kp, self.L, dtype=torch.bool)
        self.chg_sus = torch.zeros(self.Kp, self.L, dtype=DT)
        self.chg_cap = torch.zeros(self.Kp, self.L, dtype=DT)
        if ck is not None:
            for k, l, b, u in zip(np.asarray(ck), np.asarray(inst.chg_line),
                                  np.asarray(inst.chg_sus, float), np.asarray(inst.chg_cap, float)):
                self.chg[int(k), int(l)] = True
                self.chg_sus[int(k), int(l)] = float(b)
                self.chg_cap[int(k), int(l)] = float(u)
        self.gen_c2, self.gen_c1 = _t(inst.gen_c2), _t(inst.gen_c1)
        self.gen_pmin = _t(inst.gen_pmin)
        self.gen_pmax = _t(inst.gen_pmax) if gen_pmax is None else gen_pmax
        ramp = _t(inst.gen_ramp)
        self.gen_ramp = ramp
        self.is_ramp = (ramp > 0) & torch.isfinite(ramp) & torch.tensor(self.T > 1)
        self.load_d = _t(inst.load_d) if load_d is None else load_d
        self.bat_P, self.bat_dur = _t(inst.bat_P), _t(inst.bat_dur)
        self.bat_eta, self.bat_alpha = _t(inst.bat_eta), _t(inst.bat_alpha)
        d = inst.load_d
        self.load_rms = float(math.sqrt(float((_t(d) ** 2).mean()))) if self.D * self.T > 0 else 1.0

    # ---- average and residual operators (Section 2, Appendix B) ----------
    def node_sum(self, x):
        """Sum over the terminals of each node: (Kp, J, T) -> (Kp, N, T)."""
        out = torch.zeros(x.shape[0], self.N, x.shape[2], dtype=x.dtype)
        return out.index_add(1, self.term_node, x)

    def line_params(self):
        """Susceptance and capacity of every line in every contingency, [K+1][L]:
        the base values, zeroed for the N-1 outage of each contingency, with
        the listed per-contingency changes in place (Section 2.3)."""
        s = torch.where(self.chg, self.chg_sus, self.sus[None, :] * self.alive)
        c = torch.where(self.chg, self.chg_cap, self.cap[None, :] * self.alive)
        return s, c

    def avg(self, x):
        """xbar_j = (1/|n|) sum_{j' in n} x_j', returned per terminal."""
        nodes = self.node_sum(x) / self.deg[None, :, None]
        return nodes[:, self.term_node, :]

    def resid(self, x):
        return x - self.avg(x)

    def first_terminal(self):
        """Lowest-numbered terminal of every node."""
        out = torch.full((self.N,), self.J, dtype=torch.long)
        return out.scatter_reduce(0, self.term_node, torch.arange(self.J), reduce="amin")


# ---- proximal operators (Section 4.2) -----------------------------------

def prox_generator(x, rho, c2, c1, pmin, pmax):
    """argmin_p c2 p^2 + c1 p + I{pmin<=p<=pmax} + rho/2 (p - x)^2."""
    return torch.minimum(torch.maximum((rho * x - c1) / (2.0 * c2 + rho), pmin), pmax)


def prox_line(z1, z2, xi1, xi2, s, c, rho_p, rho_th, dc=None):
    """Prox of the AC line cost I{p1+p2=0} + I{|p2|<=c} + I{p2 = s (th1-th2)}.

    Returns (p1, p2, th1, th2).  Where s == 0 (an outaged line) the line
    carries no power and its phases are unconstrained.  Where dc is True (an
    HVDC link, Section 2.1: lossless power transfer within the capacity, no
    phase relation) the cost is I{p1+p2=0} + I{|p2|<=c}: the flow is the
    clipped midpoint of the two power targets and the phases keep their
    targets.
    """
    live = s > 0
    s_safe = torch.where(live, s, torch.ones_like(s))
    num = rho_p * (z2 - z1) + rho_th * (xi1 - xi2) / (2.0 * s_safe)
    den = 2.0 * rho_p + rho_th / (2.0 * s_safe * s_safe)
    p2 = torch.minimum(torch.maximum(num / den, -c), c)
    th2 = 0.5 * (xi1 + xi2) - p2 / (2.0 * s_safe)
    th1 = th2 + p2 / s_safe
    p2 = torch.where(live, p2, torch.zeros_like(p2))
    th1 = torch.where(live, th1, xi1)
    th2 = torch.where(live, th2, xi2)
    if dc is not None:
        p2dc = torch.minimum(torch.maximum(0.5 * (z2 - z1), -c), c)
        p2 = torch.where(dc, p2dc, p2)
        th1 = torch.where(dc, xi1, th1)
        th2 = torch.where(dc, xi2, th2)
    return -p2, p2, th1, th2


# ---- time-coupled devices: inner ADMM (Appendix D) ----------------------

def _diff_matrix(T):
    """(T-1) x T first difference: (Dp)_t = p_{t+1} - p_t."""
    Dm = torch.zeros(T - 1, T, dtype=DT)
    for t in range(T - 1):
        Dm[t, t] = -1.0
        Dm[t, t + 1] = 1.0
    return Dm


class RampProx:
    """Ramp-limited generators: cost c2 p^2 + c1 p with pmin <= p <= pmax
    and |p_{t+1} - p_t| <= R, evaluated by inner ADMM on the bounds A p in
    [lo, hi] with A = [I; D]."""

    def __init__(self, c2, c1, pmin, pmax, R, T):
        self.c2, self.c1, self.T = c2, c1, T
        Dm = _diff_matrix(T)
        self.A = torch.cat([torch.eye(T, dtype=DT), Dm], 0)         # (2T-1, T)
        n = c2.shape[0]
        self.lo = torch.cat([pmin, -R[:, None].expand(n, T - 1)], 1)  # (n, 2T-1)
        self.hi = torch.cat([pmax, R[:, None].expand(n, T - 1)], 1)
        self.beta = torch.zeros(n, 2 * T - 1, dtype=DT)
        self.lam = torch.zeros(n, 2 * T - 1, dtype=DT)
        self._fact = None

    def _factor(self, rho_hat, omega):
        key = (rho_hat, omega)
        if self._fact is None or self._fact[0] != key:
            AtA = self.A.T @ self.A
            M = (2.0 * self.c2 + rho_hat)[:, None, None] * torch.eye(self.T, dtype=DT) \
                + omega * AtA[None]
            self._fact = (key, torch.linalg.lu_factor(M))
        return self._fact[1]

    def __call__(self, X, rho_hat, omega, n_inner):
        LU, piv = self._factor(rho_hat, omega)
        p = None
        for _ in range(n_inner):
            # x-update: minimise c2|p|^2 + c1'p + rho_hat/2|p-X|^2 + omega/2|Ap-beta+lam|^2
            rhs = rho_hat * X - self.c1[:, None] + omega * ((self.beta - self.lam) @ self.A)
            p = torch.linalg.lu_solve(LU, piv, rhs[:, :, None])[:, :, 0]
            Ap = p @ self.A.T
            # beta-update: projection onto the bounds
            self.beta = torch.minimum(torch.maximum(Ap + self.lam, self.lo), self.hi)
            # dual update
            self.lam = self.lam + Ap - self.beta
        return p

    def rescale(self, f):
        self.lam = self.lam * f


class BatteryProx:
    """Batteries: min alpha 1'delta with p = delta - c,
    s_{t+1} = s_t + eta c_t - delta_t, s_1 = s_{T+1} = 0 and the bounds
    0 <= c, delta <= P, 0 <= s <= dur P.  Variables x = (c, delta, s) with
    s in R^{T+1}; the equalities stay in the x-update (a dense KKT solve),
    the bounds on c, delta and s_2..s_T are split off."""

    def __init__(self, P, dur, eta, alpha, T):
        n = P.shape[0]
        self.T, self.n = T, n
        self.alpha = alpha
        nx = 3 * T + 1
        self.nx = nx
        ic, idl, is_ = 0, T, 2 * T
        # equality rows: dynamics (T) then s_1 = 0, s_{T+1} = 0
        E = torch.zeros(n, T + 2, nx, dtype=DT)
        for t in range(T):
            E[:, t, is_ + t + 1] = 1.0
            E[:, t, is_ + t] = -1.0
            E[:, t, ic + t] = -eta
            E[:, t, idl + t] = 1.0
        E[:, T, is_] = 1.0
        E[:, T + 1, is_ + T] = 1.0
        self.E = E
        # split rows: c, delta, s_2..s_T
        rows = list(range(2 * T)) + [is_ + t for t in range(1, T)]
        Bs = torch.zeros(len(rows), nx, dtype=DT)
        for r, col in enumerate(rows):
            Bs[r, col] = 1.0
        self.Bs = Bs
        m = len(rows)
        self.lo = torch.zeros(n, m, dtype=DT)
        self.hi = torch.cat([P[:, None].expand(n, 2 * T),
                             (dur * P)[:, None].expand(n, T - 1)], 1)
        # p = delta - c
        self.Pmap = torch.zeros(T, nx, dtype=DT)
        for t in range(T):
            self.Pmap[t, idl + t] = 1.0
            self.Pmap[t, ic + t] = -1.0
        self.beta = torch.zeros(n, m, dtype=DT)
        self.lam = torch.zeros(n, m, dtype=DT)
        self.delta = torch.zeros(n, T, dtype=DT)
        self._fact = None

    def _factor(self, rho_hat, omega):
        key = (rho_hat, omega)
        if self._fact is None or self._fact[0] != key:
            T, n, nx = self.T, self.n, self.nx
            Q = rho_hat * (self.Pmap.T @ self.Pmap) + omega * (self.Bs.T @ self.Bs)
            K = torch.zeros(n, nx + T + 2, nx + T + 2, dtype=DT)
            K[:, :nx, :nx] = Q
            K[:, :nx, nx:] = self.E.transpose(1, 2)
            K[:, nx:, :nx] = self.E
            self._fact = (key, torch.linalg.lu_factor(K))
        return self._fact[1]

    def __call__(self, X, rho_hat, omega, n_inner):
        T = self.T
        LU, piv = self._factor(rho_hat, omega)
        lin = torch.zeros(self.n, self.nx, dtype=DT)
        lin[:, T:2 * T] = self.alpha[:, None]
        p = None
        for _ in range(n_inner):
            # x-update: min alpha'delta + rho_hat/2|Pmap x - X|^2
            #              + omega/2|Bs x - beta + lam|^2  s.t. E x = 0
            g = rho_hat * (X @ self.Pmap) + omega * ((self.beta - self.lam) @ self.Bs) - lin
            rhs = torch.cat([g, torch.zeros(self.n, T + 2, dtype=DT)], 1)
            sol = torch.linalg.lu_solve(LU, piv, rhs[:, :, None])[:, :, 0]
            x = sol[:, :self.nx]
            Bx = x @ self.Bs.T
            self.beta = torch.minimum(torch.maximum(Bx + self.lam, self.lo), self.hi)
            self.lam = self.lam + Bx - self.beta
            p = x @ self.Pmap.T
            self.delta = x[:, T:2 * T]
        return p

    def rescale(self, f):
        self.lam = self.lam * f


# ---- the message-passing solver (Section 3.2) ---------------------------

@dataclass
class Residual:
    iter: int
    primal_p: float      # ||pbar||
    primal_th: float     # ||theta tilde||
    dual_p: float        # rho_p ||ptilde' - ptilde||
    dual_th: float       # rho_theta ||thetabar' - thetabar||
    rms_primal: float
    rms_dual: float
    threshold: float
    objective: float
    rho_p: float
    rho_theta: float
    converged: bool


class Solver:
    """Runs the message-passing iteration from the all-zero start, or from
    an iterate exported by another run (init, see export_state)."""

    def __init__(self, inst, opt: Optional[Options] = None, load_d=None, line_cap=None,
                 gen_pmax=None, init: Optional[Dict] = None):
        self.net = net = Network(inst, load_d=load_d, line_cap=line_cap, gen_pmax=gen_pmax)
        self.opt = opt or Options()
        self.rho_p = float(self.opt.rho_p)
        self.rho_th = float(self.opt.rho_theta)
        Kp, J, T = net.Kp, net.J, net.T
        z = lambda: torch.zeros(Kp, J, T, dtype=DT)
        self.p, self.th, self.u, self.v = z(), z(), z(), z()
        self.pbar, self.thbar = z(), z()
        self.iter = 0
        L, G, D = net.L, net.G, net.D
        self.sl_gen = slice(2 * L, 2 * L + G)
        self.sl_load = slice(2 * L + G, 2 * L + G + D)
        self.sl_bat = slice(2 * L + G + D, J)
        ramp_idx = torch.nonzero(net.is_ramp).flatten()
        plain_idx = torch.nonzero(~net.is_ramp).flatten()
        self.ramp_idx, self.plain_idx = ramp_idx, plain_idx
        self.ramp = None
        if len(ramp_idx) > 0:
            self.ramp = RampProx(net.gen_c2[ramp_idx], net.gen_c1[ramp_idx],
                                 net.gen_pmin[ramp_idx], net.gen_pmax[ramp_idx],
                                 net.gen_ramp[ramp_idx], T)
        self.bat = None
        if net.B > 0:
            self.bat = BatteryProx(net.bat_P, net.bat_dur, net.bat_eta, net.bat_alpha, T)
        scale = net.load_rms if self.opt.eps_relative else 1.0
        self.eps_eff = self.opt.eps * scale
        self.history: List[Residual] = []
        a = float(self.opt.alpha)
        if not 1.0 <= a < 2.0:
            raise ValueError("the relaxation parameter alpha must lie in [1, 2)")
        self.relaxed = a != 1.0 or self.opt.explicit_copies
        self.z, self.xi = z(), z()       # duplicate variables (relaxed form only)
        if init is not None:
            self.load_state(init)

    # -- warm start (Section 3.4) ---------------------------------------------
    _STATE = ("p", "th", "u", "v", "pbar", "thbar", "z", "xi")

    def export_state(self) -> Dict:
        """The whole iterate: per-terminal tensors, the inner ADMM state of
        ramp generators and batteries, and the penalties (copies)."""
        out = {k: getattr(self, k).clone() for k in self._STATE}
        out["rho_p"], out["rho_th"] = self.rho_p, self.rho_th
        if self.ramp is not None:
            out["ramp"] = (self.ramp.beta.clone(), self.ramp.lam.clone())
        if self.bat is not None:
            out["bat"] = (self.bat.beta.clone(), self.bat.lam.clone(), self.bat.delta.clone())
        return out

    def load_state(self, st: Dict):
        """Continues from an exported iterate of a network with the same
        structure (terminal order, contingency count, horizon and device
        classes); the problem data may differ.  The iteration count restarts
        at zero."""
        for k in self._STATE:
            if tuple(st[k].shape) != tuple(getattr(self, k).shape):
                raise ValueError(f"state {k} has shape {tuple(st[k].shape)}, "
                                 f"this network needs {tuple(getattr(self, k).shape)}")
            setattr(self, k, st[k].detach().clone().to(DT))
        self.rho_p, self.rho_th = float(st["rho_p"]), float(st["rho_th"])
        for name in ("ramp", "bat"):
            dev = getattr(self, name)
            if (dev is None) != (st.get(name) is None):
                raise ValueError(f"{name} devices differ between the state and this network")
            if dev is not None:
                parts = st[name]
                if tuple(parts[0].shape) != tuple(dev.beta.shape):
                    raise ValueError(f"{name} inner state has another shape")
                dev.beta, dev.lam = parts[0].clone(), parts[1].clone()
                if name == "bat":
                    dev.delta = parts[2].clone()
        self.iter = 0
        self.history = []

    # -- one iteration ------------------------------------------------------
    def step(self):
        net, opt = self.net, self.opt
        L, Kp, T = net.L, net.Kp, net.T
        rp, rt = self.rho_p, self.rho_th
        p, th, u, v = self.p, self.th, self.u, self.v
        pbar, thbar = self.pbar, self.thbar
        ptil = p - pbar
        a = float(opt.alpha)

        # step 1: contingency prox on the lines, per contingency k, at the
        # targets z - u and xi - v (z = ptilde and xi = thetabar in the
        # message-passing form; explicit copies when relaxed, Section 3.6)
        if self.relaxed:
            x = self.z - u
            y = self.xi - v
        else:
            x = ptil - u
            y = thbar - v
        s, c = net.line_params()
        s, c = s[:, :, None], c[:, :, None]
        p1, p2, th1, th2 = prox_line(x[:, :L], x[:, L:2 * L], y[:, :L], y[:, L:2 * L],
                                     s, c, rp, rt, net.dc[None, :, None].expand_as(s))

        # step 2: non-contingency prox with penalty (K+1) rho at the
        # contingency-averaged targets
        rho_hat = Kp * rp
        if self.relaxed:
            X = x.mean(0)[2 * L:]                  # avg_k(z_k - u_k)
            Y = y.mean(0)[2 * L:]                  # avg_k(xi_k - v_k)
        else:
            X = (p - (pbar + u)).mean(0)[2 * L:]   # p - avg_k(pbar_k + u_k)
            Y = (thbar - v).mean(0)[2 * L:]        # avg_k(thbar_k - v_k)
        pnc = torch.zeros(net.Jnc, T, dtype=DT)
        G, D = net.G, net.D
        Xg = X[:G]
        pg = torch.zeros(G, T, dtype=DT)
        if len(self.plain_idx) > 0:
            i = self.plain_idx
            pg = pg.index_copy(0, i, prox_generator(Xg[i], rho_hat, net.gen_c2[i, None],
                                                    net.gen_c1[i, None], net.gen_pmin[i],
                                                    net.gen_pmax[i]))
        if self.ramp is not None:
            omega = opt.inner_omega_scale * rho_hat
            pg = pg.index_copy(0, self.ramp_idx,
                               self.ramp(Xg[self.ramp_idx], rho_hat, omega, opt.inner_iters))
        pl = -net.load_d
        parts = [pg, pl]
        if self.bat is not None:
            omega = opt.inner_omega_scale * rho_hat
            parts.append(self.bat(X[G + D:], rho_hat, omega, opt.inner_iters))
        pnc = torch.cat(parts, 0)
        thnc = Y

        p_new = torch.cat([p1, p2, pnc[None].expand(Kp, -1, -1)], 1)
        th_new = torch.cat([th1, th2, thnc[None].expand(Kp, -1, -1)], 1)

        # step 3: averages and scaled price updates
        pbar_new = net.avg(p_new)
        thbar_new = net.avg(th_new)
        ptil_new = p_new - pbar_new
        if self.relaxed:
            z_new = a * ptil_new + (1.0 - a) * self.z
            xi_new = a * thbar_new + (1.0 - a) * self.xi
            u_new = u + a * pbar_new
            v_new = v + a * (th_new - thbar_new)
        else:
            u_new = u + pbar_new
            v_new = v + (th_new - thbar_new)

        # residuals (Section 3.3)
        r_pp = torch.sqrt((pbar_new ** 2).sum())
        r_pt = torch.sqrt(((th_new - thbar_new) ** 2).sum())
        if self.relaxed:
            r_dp = rp * torch.sqrt(((z_new - self.z) ** 2).sum())
            r_dt = rt * torch.sqrt(((xi_new - self.xi) ** 2).sum())
            self.z, self.xi = z_new, xi_new
        else:
            r_dp = rp * torch.sqrt(((ptil_new - ptil) ** 2).sum())
            r_dt = rt * torch.sqrt(((thbar_new - thbar) ** 2).sum())
        norm = math.sqrt(2.0 * net.J * T * Kp)
        rms_pri = float(torch.sqrt(r_pp ** 2 + r_pt ** 2)) / norm
        rms_dual = float(torch.sqrt(r_dp ** 2 + r_dt ** 2)) / norm

        self.p, self.th, self.u, self.v = p_new, th_new, u_new, v_new
        self.pbar, self.thbar = pbar_new, thbar_new
        self.iter += 1
        converged = max(rms_pri, rms_dual) <= self.eps_eff and self.iter >= opt.min_iter
        res = Residual(self.iter, float(r_pp), float(r_pt), float(r_dp), float(r_dt),
                       rms_pri, rms_dual, self.eps_eff, float(self.objective()),
                       rp, rt, converged)

        # adaptive penalty (Section 3.5), after iterations adapt_every, 2 adapt_every, ...
        if opt.adapt_every > 0 and self.iter % opt.adapt_every == 0:
            new_p = self._adapt(self.rho_p, float(r_pp), float(r_dp))
            new_t = self._adapt(self.rho_th, float(r_pt), float(r_dt))
            if new_p != self.rho_p:
                f = self.rho_p / new_p
                self.u = self.u * f
                if self.ramp is not None:
                    self.ramp.rescale(f)      # omega scales with rho_p
                if self.bat is not None:
                    self.bat.rescale(f)
                self.rho_p = new_p
            if new_t != self.rho_th:
                self.v = self.v * (self.rho_th / new_t)
                self.rho_th = new_t
        self.history.append(res)
        return res

    def _adapt(self, rho, r_primal, r_dual):
        mu, gamma = self.opt.mu, self.opt.gamma
        if r_primal > mu * r_dual:
            return rho * gamma
        if r_dual > mu * r_primal:
            return rho / gamma
        return rho

    def run(self, n_iters):
        for _ in range(n_iters):
            self.step()
        return self.history[-1] if self.history else None

    def solve(self):
        while self.iter < self.opt.max_iter:
            r = self.step()
            if r.converged:
                return r
        return self.history[-1]

    # -- outputs ------------------------------------------------------------
    def objective(self):
        """sum_g (c2 p^2 + c1 p) + sum_b alpha sum_t delta_t (line cost 0)."""
        net = self.net
        L, G = net.L, net.G
        pg = self.p[0, 2 * L:2 * L + G]
        obj = (net.gen_c2[:, None] * pg ** 2 + net.gen_c1[:, None] * pg).sum()
        if self.bat is not None:
            obj = obj + (net.bat_alpha[:, None] * self.bat.delta).sum()
        return obj

    def dispatch(self):
        """Non-contingency schedules p [Jnc, T] (generators, loads, batteries)."""
        return self.p[0, 2 * self.net.L:]

    def lmp(self):
        """Locational prices -rho_p * sum_k u_k per node [N, T]."""
        net = self.net
        # u is node-constant: take it from any terminal of each node
        first = net.first_terminal()
        un = self.u[:, first, :]
        return -self.rho_p * un.sum(0)

    def canonical_state(self) -> Dict[str, torch.Tensor]:
        """State in the per-line / per-node form used for GPU parity.

        P = p2 (power injected at the to node), TH1, TH2 [K+1, L, T];
        V1, V2 line-terminal phase duals [K+1, L, T]; U, PBAR, THBAR per node
        [K+1, N, T]; p, th of the non-contingency devices [Jnc, T]; VNC the
        contingency average of their phase duals [Jnc, T].
        """
        net = self.net
        L = net.L
        first = net.first_terminal()
        return dict(
            P=self.p[:, L:2 * L], TH1=self.th[:, :L], TH2=self.th[:, L:2 * L],
            V1=self.v[:, :L], V2=self.v[:, L:2 * L],
            U=self.u[:, first], PBAR=self.pbar[:, first], THBAR=self.thbar[:, first],
            PNC=self.p[0, 2 * L:], THNC=self.th[0, 2 * L:],
            VNC=self.v[:, 2 * L:].mean(0),
        )
