"""Seeded synthetic contingency-constrained DC OPF instances.

This module only builds problem data (grids, devices, loads, outages); it
holds none of the message-passing arithmetic, and both the HIP path and the
CPU oracle take its output as plain arrays.

The paper's workloads come from the PyPSA-USA Western Interconnect (Section 5
and Appendix E), which is not available here.  Synthetic grids with the same
structure stand in for it: sparse meshed transmission grids with locality,
quadratic-cost generators with box and ramp limits, batteries, fixed loads
with a daily profile, and N-1 single-line outages (Section 2.3).

Generation recipe (every random draw has its own named PCG64 sub-stream):

* topology: nodes uniform in the unit square; a random-weight minimum
  spanning tree of the 6-nearest-neighbour graph gives a spanning tree with
  locality, then extra lines are drawn uniformly from the remaining 6-NN
  pairs.  Nodes are relabelled in Hilbert-curve order and lines sorted by
  (from, to) so that grid neighbours are memory neighbours;
* lines: susceptance U[5, 20], capacity U[0.5, 2];
* generators on distinct nodes: pmax U[1, 3], c2 U[0.01, 0.1], c1 U[10, 50],
  pmin 0, ramp limit 0.3 pmax when T > 1;
* loads on distinct nodes: base U[0.1, 0.5]; for T > 1 the demand is
  base * (1 + 0.3 sin(2 pi ((t mod 24) - 8) / 24)) * U[0.8, 1.2];
* batteries on distinct nodes: energy E U[1, 4], power P = E/4,
  duration 4, efficiency 0.95, discharge cost 1;
* contingencies: K distinct non-bridge lines (so every post-outage grid
  stays connected and flows are unique) that a generator redispatch can
  idle in every period (below);
* feasibility: pmax is scaled so that total capacity is at least 1.25x the
  peak total load.  The reference dispatch starts with generators
  proportional to pmax (batteries idle).  Non-bridge lines are then tried
  in a seeded random order, and a line becomes an outage if the dispatch,
  corrected to carry no power on it and on every outage already taken
  (least change in the metric weighted by pmax, so that the balance and
  the earlier outages stay exact), keeps every generator within
  [0.01 pmax, 1.5 pmax] and within 0.99 of its ramp limit; pmax is raised
  to 1/0.99 of a dispatch above it and the ramp limit is 0.3 pmax.  Every
  line capacity is then raised to 1.1x the largest base or post-outage
  flow of that dispatch (DC power flow).
  Why: in the problem of Section 2.3 the power and the phase of every
  device node are shared by all contingencies.  Where most nodes host a
  device (as in these grids and the paper's), the flows of the lines
  between them are then the same in every contingency, so a feasible point
  needs (nearly) zero base flow on each outaged line; a capacity rule for
  free post-outage phases (the textbook N-1 problem) does not provide one,
  and grids with uniformly drawn outages are in general infeasible.  The
  reference dispatch above carries no power on the outaged lines, so its
  base phases, used unchanged in every contingency, satisfy every
  contingency's balance and every capacity: the instance is feasible for
  the problem as posed (and for the textbook N-1 problem).
  Where fewer than K lines pass (small grids: K outages and the balance
  need at least K + 1 generators), the remaining outages are drawn
  uniformly from the other candidates and the instance is certified for
  free post-outage phases only (`meta["K_idle"]` < K); `outage_rule=
  "idle_only"` keeps only the idle lines instead (fewer contingencies), and
  `outage_rule="uniform"` draws all K uniformly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Instance:
    """One contingency-constrained DC OPF problem (device-node model).

    Node ids are 0..N-1.  Line l connects terminal 1 at node line_from[l] to
    terminal 2 at node line_to[l].  Contingency k in 1..K removes line
    outage[k-1] (an outage id of -1 means the contingency changes nothing).
    Per-time arrays are [device][t] row-major.  Fixed load demands are
    stored positive; the load's injection is minus the demand.
    """
    name: str
    N: int
    T: int
    K: int
    line_from: np.ndarray
    line_to: np.ndarray
    line_sus: np.ndarray
    line_cap: np.ndarray
    outage: np.ndarray
    gen_node: np.ndarray
    gen_c2: np.ndarray
    gen_c1: np.ndarray
    gen_pmin: np.ndarray
    gen_pmax: np.ndarray
    gen_ramp: np.ndarray
    load_node: np.ndarray
    load_d: np.ndarray
    bat_node: np.ndarray
    bat_P: np.ndarray
    bat_dur: np.ndarray
    bat_eta: np.ndarray
    bat_alpha: np.ndarray
    line_kind: Optional[np.ndarray] = None  # [L] 0 = AC line, 1 = DC link; None = all AC
    # per-contingency line parameters (Section 2.3): contingency chg_k[i] gives
    # line chg_line[i] susceptance chg_sus[i] and capacity chg_cap[i]
    # (susceptance 0: the line is out); None = the N-1 outages only
    chg_k: Optional[np.ndarray] = None
    chg_line: Optional[np.ndarray] = None
    chg_sus: Optional[np.ndarray] = None
    chg_cap: Optional[np.ndarray] = None
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.line_from.shape[0])

    @property
    def G(self) -> int:
        return int(self.gen_node.shape[0])

    @property
    def D(self) -> int:
        return int(self.load_node.shape[0])

    @property
    def B(self) -> int:
        return int(self.bat_node.shape[0])

    @property
    def J(self) -> int:
        """Number of terminals: two per line, one per other device."""
        return 2 * self.L + self.G + self.D + self.B

    def load_rms(self) -> float:
        """Root mean square of the demand over all loads and times."""
        if self.load_d.size == 0:
            return 1.0
        return float(np.sqrt(np.mean(self.load_d.astype(np.float64) ** 2)))

    def copy(self) -> "Instance":
        return dataclasses.replace(
            self, **{f.name: (getattr(self, f.name).copy()
                              if isinstance(getattr(self, f.name), np.ndarray)
                              else getattr(self, f.name))
                     for f in dataclasses.fields(self)})


# --------------------------------------------------------------------------
# graph helpers


def _hilbert_index(x: np.ndarray, y: np.ndarray, order: int = 16) -> np.ndarray:
    """Index along a Hilbert curve of the 2^order grid (vectorised)."""
    n = 1 << order
    xi = np.clip((x * (n - 1)).astype(np.int64), 0, n - 1)
    yi = np.clip((y * (n - 1)).astype(np.int64), 0, n - 1)
    d = np.zeros_like(xi)
    s = n >> 1
    while s > 0:
        rx = ((xi & s) > 0).astype(np.int64)
        ry = ((yi & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = ry == 0
        swap_x = np.where(flip & (rx == 1), s - 1 - xi, xi)
        swap_y = np.where(flip & (rx == 1), s - 1 - yi, yi)
        xi = np.where(flip, swap_y, xi)
        yi = np.where(flip, swap_x, yi)
        s >>= 1
    return d


def _components(n: int, edges: np.ndarray) -> np.ndarray:
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    if edges.shape[0] == 0:
        return np.arange(n)
    m = coo_matrix((np.ones(edges.shape[0]), (edges[:, 0], edges[:, 1])), shape=(n, n))
    _, lab = connected_components(m, directed=False)
    return lab


def bridges(n: int, frm: np.ndarray, to: np.ndarray) -> np.ndarray:
    """Boolean mask of bridge lines (iterative Tarjan low-link DFS)."""
    L = frm.shape[0]
    adj: List[List[tuple]] = [[] for _ in range(n)]
    for l in range(L):
        a, b = int(frm[l]), int(to[l])
        adj[a].append((b, l))
        adj[b].append((a, l))
    disc = np.full(n, -1, dtype=np.int64)
    low = np.zeros(n, dtype=np.int64)
    is_bridge = np.zeros(L, dtype=bool)
    timer = 0
    for root in range(n):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, 0)]  # node, parent edge, next neighbour position
        while stack:
            v, pe, i = stack[-1]
            if i < len(adj[v]):
                stack[-1] = (v, pe, i + 1)
                w, e = adj[v][i]
                if e == pe:
                    continue
                if disc[w] < 0:
                    disc[w] = low[w] = timer
                    timer += 1
                    stack.append((w, e, 0))
                else:
                    low[v] = min(low[v], disc[w])
            else:
                stack.pop()
                if stack:
                    u = stack[-1][0]
                    low[u] = min(low[u], low[v])
                    if low[v] > disc[u]:
                        is_bridge[pe] = True
    return is_bridge


def _make_topology(rng_topo: np.random.Generator, N: int, L: int):
    """Spanning tree with locality plus extra lines from the 6-NN pairs."""
    from scipy.spatial import cKDTree
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    assert L >= N - 1, "need at least a spanning tree"
    xy = rng_topo.random((N, 2))
    order = np.argsort(_hilbert_index(xy[:, 0], xy[:, 1]), kind="stable")
    xy = xy[order]  # nodes relabelled in Hilbert order
    kq = min(7, N)
    _, nb = cKDTree(xy).query(xy, k=kq)
    pairs = set()
    for i in range(N):
        for j in nb[i, 1:]:
            a, b = (i, int(j)) if i < j else (int(j), i)
            if a != b:
                pairs.add((a, b))
    pairs = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
    w = rng_topo.random(pairs.shape[0]) + 1e-3
    m = coo_matrix((w, (pairs[:, 0], pairs[:, 1])), shape=(N, N))
    mst = minimum_spanning_tree(m).tocoo()
    tree = set((min(a, b), max(a, b)) for a, b in zip(mst.row.tolist(), mst.col.tolist()))
    # the 6-NN graph may be disconnected: join components by nearest pairs
    edges = np.array(sorted(tree), dtype=np.int64).reshape(-1, 2)
    lab = _components(N, edges)
    while len(np.unique(lab)) > 1:
        c0 = lab == lab[0]
        ia = np.nonzero(c0)[0]
        ib = np.nonzero(~c0)[0]
        tb = cKDTree(xy[ib])
        dist, jj = tb.query(xy[ia], k=1)
        a = int(ia[np.argmin(dist)])
        b = int(ib[jj[np.argmin(dist)]])
        tree.add((min(a, b), max(a, b)))
        edges = np.array(sorted(tree), dtype=np.int64).reshape(-1, 2)
        lab = _components(N, edges)
    rest = [tuple(p) for p in pairs.tolist() if tuple(p) not in tree]
    n_extra = L - len(tree)
    if n_extra > len(rest):
        raise ValueError(f"6-NN graph has only {len(rest)} spare pairs, need {n_extra}")
    pick = rng_topo.choice(len(rest), size=n_extra, replace=False) if n_extra > 0 else []
    all_edges = sorted(list(tree) + [rest[i] for i in pick])
    e = np.array(all_edges, dtype=np.int64).reshape(-1, 2)
    return xy, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def _dc_flows(N, frm, to, sus, inj):
    """DC power-flow line flows (from -> to) for injections inj [N, T]."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.linalg import splu
    L = frm.shape[0]
    rows = np.concatenate([frm, to, frm, to])
    cols = np.concatenate([frm, to, to, frm])
    vals = np.concatenate([sus, sus, -sus, -sus])
    Bm = coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsc()
    red = Bm[1:, 1:].tocsc()  # node 0 is the angle reference
    lu = splu(red)
    th = np.zeros((N, inj.shape[1]))
    if N > 1:
        th[1:] = lu.solve(np.ascontiguousarray(inj[1:]))
    flows = sus[:, None] * (th[frm] - th[to])
    return flows, lu


def _raise_caps_for_n1(N, frm, to, sus, cap, outage, inj):
    """Raise capacities to 1.1x the worst base/post-outage reference flow."""
    flows, lu = _dc_flows(N, frm, to, sus, inj)
    worst = np.abs(flows).max(axis=1)
    scale = max(1.0, float(np.abs(flows).max())) if flows.size else 1.0
    for o in outage:
        if o < 0 or np.abs(flows[o]).max() <= 1e-9 * scale:
            continue  # an idle line's outage leaves every flow as it is
        rhs = np.zeros(N)
        rhs[frm[o]] += 1.0
        rhs[to[o]] -= 1.0
        x = np.zeros(N)
        if N > 1:
            x[1:] = lu.solve(rhs[1:])
        ptdf = sus * (x[frm] - x[to])  # flow change per unit transfer f_o -> h_o
        denom = 1.0 - ptdf[o]
        lodf = ptdf / denom
        lodf[o] = -1.0
        post = flows + lodf[:, None] * flows[o][None, :]
        worst = np.maximum(worst, np.abs(post).max(axis=1))
    new_cap = np.maximum(cap, 1.1 * worst)
    return new_cap, float(np.mean(new_cap > cap))


def _idle_outages(N, frm, to, sus, gen_node, load_node, demand, pmax1, disp, order, K,
                  use_ramp):
    """Greedy choice of up to K outages from `order` that a generator
    redispatch idles in every period (recipe in the module docstring).

    Returns (outages, dispatch [G, T], pmax [G]).  The correction for each
    new line is the pmax-weighted least-norm change that zeroes its flow
    while keeping the balance and the earlier zero flows: with A the
    accepted constraint rows over generator injections (first row: the
    balance) and W = diag(pmax), the direction is g = W a - W A^T M^-1 A W a
    with M = A W A^T, which A maps to zero."""
    G, T = gen_node.shape[0], demand.shape[1]
    _, lu = _dc_flows(N, frm, to, sus, np.zeros((N, 1)))
    W = np.asarray(pmax1, dtype=np.float64)
    A = np.ones((1, G))
    Minv = np.array([[1.0 / W.sum()]])
    p = disp.copy()
    pmax = W.copy()
    taken = []
    xs = {}
    for i, l in enumerate(order):
        if len(taken) == K:
            break
        if l not in xs:  # sensitivities of the next candidates, one solve per block
            blk = order[i:i + 64]
            rhs = np.zeros((N, len(blk)))
            rhs[frm[blk], np.arange(len(blk))] += 1.0
            rhs[to[blk], np.arange(len(blk))] -= 1.0
            x = np.zeros((N, len(blk)))
            if N > 1:
                x[1:] = lu.solve(np.ascontiguousarray(rhs[1:]))
            xs = {int(c): x[:, j] for j, c in enumerate(blk)}
        s_n = sus[l] * xs[int(l)]  # flow on l per unit injected at each node (out at node 0)
        a = s_n[gen_node]
        flow = a @ p - s_n[load_node] @ demand  # [T]
        Wa = W * a
        m = A @ Wa
        Mm = Minv @ m
        g = Wa - W * (A.T @ Mm)
        sc = float(a @ g)
        if not sc > 1e-9 * float(a @ Wa):
            continue  # the earlier rows already fix this flow
        q = p - g[:, None] * (flow[None, :] / sc)
        if not (np.all(q >= 0.01 * pmax[:, None]) and np.all(q <= 1.5 * pmax[:, None])):
            continue
        if use_ramp and T > 1:
            pm = np.maximum(pmax, q.max(axis=1) / 0.99)
            if not np.all(np.abs(np.diff(q, axis=1)) <= 0.99 * 0.3 * pm[:, None]):
                continue
        p = q
        taken.append(int(l))
        # bordered inverse of M with the new row a appended to A
        Minv = np.block([[Minv + np.outer(Mm, Mm) / sc, -Mm[:, None] / sc],
                         [-Mm[None, :] / sc, np.array([[1.0 / sc]])]])
        A = np.vstack([A, a])
    pmax = np.maximum(pmax, p.max(axis=1) / 0.99) if T > 0 else pmax
    return np.sort(np.asarray(taken, dtype=np.int32)), p, pmax


def make_instance(name: str, N: int, L: int, G: int, D: int, B: int, T: int, K: int,
                  seed: int, ramp: Optional[bool] = None, outage_rule: str = "idle") -> Instance:
    """Build one seeded synthetic instance (recipe in the module docstring).

    outage_rule: "idle" (outages that a redispatch idles, topped up with
    uniform draws if too few exist), "idle_only" (only those: K may shrink,
    `meta["K_requested"]` keeps the request) or "uniform"."""
    if outage_rule not in ("idle", "idle_only", "uniform"):
        raise ValueError(f"unknown outage_rule {outage_rule!r}")
    ss = np.random.SeedSequence(seed)
    topo, lines, gens, loads, bats, cont = [np.random.Generator(np.random.PCG64(s))
                                            for s in ss.spawn(6)]
    xy, frm, to = _make_topology(topo, N, L)
    sus = lines.uniform(5.0, 20.0, L)
    cap = lines.uniform(0.5, 2.0, L)

    gen_node = np.sort(gens.choice(N, size=G, replace=False)).astype(np.int32)
    pmax1 = gens.uniform(1.0, 3.0, G)
    c2 = gens.uniform(0.01, 0.1, G)
    c1 = gens.uniform(10.0, 50.0, G)

    load_node = np.sort(loads.choice(N, size=D, replace=False)).astype(np.int32)
    base = loads.uniform(0.1, 0.5, D)
    if T > 1:
        t = np.arange(T)
        shape = 1.0 + 0.3 * np.sin(2.0 * np.pi * ((t % 24) - 8) / 24.0)
        noise = loads.uniform(0.8, 1.2, (D, T))
        demand = base[:, None] * shape[None, :] * noise
    else:
        demand = base[:, None].copy()

    bat_node = np.sort(bats.choice(N, size=B, replace=False)).astype(np.int32)
    energy = bats.uniform(1.0, 4.0, B)
    bat_P = 0.25 * energy
    bat_dur = np.full(B, 4.0)
    bat_eta = np.full(B, 0.95)
    bat_alpha = np.full(B, 1.0)

    # contingency candidates: distinct non-bridge lines
    br = bridges(N, frm, to)
    cand = np.nonzero(~br)[0]
    if K > len(cand):
        raise ValueError(f"only {len(cand)} non-bridge lines for K={K}")

    # feasibility rule
    peak = demand.sum(axis=0).max() if D > 0 else 0.0
    scale = max(1.0, 1.25 * peak / max(pmax1.sum(), 1e-12))
    pmax1 = pmax1 * scale
    use_ramp = (T > 1) if ramp is None else ramp
    total = demand.sum(axis=0)  # [T]
    disp = pmax1[:, None] * (total / pmax1.sum())[None, :]
    K_req = K
    if outage_rule != "uniform" and K > 0:
        order = cont.permutation(cand)
        outage, disp, pmax1 = _idle_outages(N, frm, to, sus, gen_node, load_node, demand,
                                            pmax1, disp, order, K, use_ramp)
        K_idle = int(outage.shape[0])
        if outage_rule == "idle_only":
            K = K_idle
        elif K_idle < K:
            rest = np.setdiff1d(cand, outage)
            more = cont.choice(rest, size=K - K_idle, replace=False)
            outage = np.sort(np.r_[outage, more]).astype(np.int32)
    else:
        outage = np.sort(cont.choice(cand, size=K, replace=False)).astype(np.int32)
        K_idle = 0
    pmax = np.repeat(pmax1[:, None], T, axis=1)
    pmin = np.zeros((G, T))
    gen_ramp = 0.3 * pmax1 if use_ramp else np.zeros(G)
    inj = np.zeros((N, T))
    np.add.at(inj, gen_node, disp)
    np.subtract.at(inj, load_node, demand)
    cap, frac = _raise_caps_for_n1(N, frm, to, sus, cap, outage, inj)

    return Instance(
        name=name, N=N, T=T, K=K,
        line_from=frm.astype(np.int32), line_to=to.astype(np.int32),
        line_sus=sus, line_cap=cap, outage=outage,
        gen_node=gen_node, gen_c2=c2, gen_c1=c1, gen_pmin=pmin, gen_pmax=pmax,
        gen_ramp=gen_ramp,
        load_node=load_node, load_d=demand,
        bat_node=bat_node, bat_P=bat_P, bat_dur=bat_dur, bat_eta=bat_eta,
        bat_alpha=bat_alpha,
        meta={"seed": seed, "frac_lines_raised": frac, "capacity_scale": scale,
              "K_requested": K_req, "K_idle": K_idle, "outage_rule": outage_rule,
              # the reference dispatch [G, T] (batteries idle) that certifies
              # feasibility: N-1 with free post-outage phases always, and with
              # the device phases shared by all contingencies when every
              # outage is idle (K_idle == K: no power on any outaged line)
              "ref_dispatch": disp},
    )


# Named workloads.  Sizes follow the paper's experiment families: a small
# parity case, a 500-node day-ahead case with N-1 outages (Section 5.3), the
# >5e8-variable scale of Section 5.4, a batch of uneven instances (Section
# 5.6) and the 500-node differentiation case (Section 5.5).
CONFIGS = {
    "tiny": dict(N=14, L=19, G=5, D=11, B=0, T=1, K=0, seed=14),
    "medium": dict(N=500, L=700, G=100, D=400, B=20, T=24, K=50, seed=500),
    "large": dict(N=10000, L=13000, G=2000, D=8000, B=500, T=96, K=200, seed=10000),
    "diff": dict(N=500, L=700, G=100, D=400, B=20, T=24, K=20, seed=2024),
}


def config(name: str, **over) -> Instance:
    """Instance for a named workload; keyword overrides replace sizes."""
    kw = dict(CONFIGS[name])
    kw.update(over)
    return make_instance(name, **kw)


def batched_configs(n: int = 64, seed: int = 64) -> List[dict]:
    """Size draws for the batch of uneven instances."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    out = []
    for i in range(n):
        N = int(round(math.exp(rng.uniform(math.log(100), math.log(2000)))))
        T = int(rng.choice([1, 24, 48]))
        K = int(rng.integers(0, 31))
        out.append(dict(N=N, L=int(round(1.4 * N)), G=int(round(0.2 * N)),
                        D=int(round(0.8 * N)), B=int(round(0.04 * N)), T=T, K=K,
                        seed=seed * 1000 + i))
    return out


def batched(n: int = 64, seed: int = 64) -> List[Instance]:
    """The batch of uneven instances; each keeps only outages that a
    redispatch idles, so every instance is feasible with shared device
    phases (a few get fewer contingencies than drawn)."""
    return [make_instance(f"batch{i}", outage_rule="idle_only", **kw)
            for i, kw in enumerate(batched_configs(n, seed))]


def two_node(d: float = 1.0, c2=(0.5, 0.25), c1=(1.0, 2.0), pmax=(5.0, 5.0),
             sus: float = 1.0, cap: float = 10.0, T: int = 1) -> Instance:
    """Two nodes, one line: generator 1 at node 0; generator 2 and a load at node 1."""
    f = lambda v: np.asarray(v, dtype=np.float64)
    return Instance(
        name="two_node", N=2, T=T, K=0,
        line_from=np.array([0], np.int32), line_to=np.array([1], np.int32),
        line_sus=f([sus]), line_cap=f([cap]), outage=np.zeros(0, np.int32),
        gen_node=np.array([0, 1], np.int32), gen_c2=f(c2), gen_c1=f(c1),
        gen_pmin=np.zeros((2, T)), gen_pmax=np.repeat(f(pmax)[:, None], T, 1),
        gen_ramp=np.zeros(2),
        load_node=np.array([1], np.int32), load_d=np.full((1, T), float(d)),
        bat_node=np.zeros(0, np.int32), bat_P=f([]), bat_dur=f([]), bat_eta=f([]),
        bat_alpha=f([]), meta={},
    )


def with_curtailable_loads(inst: Instance, cost: float = 500.0) -> Instance:
    """The same network with every fixed load replaced by a curtailable one
    (Section 2.1: a generator with pmin = -d_t < pmax = 0 and linear cost;
    serving the demand in full is worth `cost` per unit).  Loads become the
    last generators; the instance has no fixed loads."""
    import dataclasses as _dc
    G, D, T = len(inst.gen_node), len(inst.load_node), int(inst.T)
    d = np.asarray(inst.load_d, float).reshape(D, T)
    return _dc.replace(
        inst,
        gen_node=np.r_[inst.gen_node, inst.load_node].astype(np.int32),
        gen_c2=np.r_[inst.gen_c2, np.zeros(D)],
        gen_c1=np.r_[inst.gen_c1, np.full(D, cost)],
        gen_pmin=np.r_[np.asarray(inst.gen_pmin, float).reshape(G, T), -d],
        gen_pmax=np.r_[np.asarray(inst.gen_pmax, float).reshape(G, T), np.zeros((D, T))],
        gen_ramp=np.r_[inst.gen_ramp, np.full(D, np.inf)],
        load_node=np.zeros(0, np.int32),
        load_d=np.zeros((0, T)),
    )


def with_dc_links(inst: Instance, count: int = 3, seed: int = 0, outage_first: bool = True,
                  cap=(1.0, 3.0)) -> Instance:
    """The same network plus `count` HVDC links (Section 2.1; the paper's
    western-interconnect case has 3 among about 1150 lines) appended after
    the AC lines.  Each joins two seed-chosen nodes at least N/4 apart in the
    Hilbert node order (long-distance links), with capacity U[cap]; a DC
    link's susceptance is ignored (stored as 10).  With outage_first and
    K >= 1, contingency 1 removes the first DC link instead of its AC line.
    Every existing N-1-feasible dispatch stays feasible with the links idle."""
    import dataclasses as _dc
    rng = np.random.default_rng([seed, 0xDC])
    N, L = int(inst.N), len(inst.line_from)
    frm, to = [], []
    seen = set(zip(np.asarray(inst.line_from).tolist(), np.asarray(inst.line_to).tolist()))
    while len(frm) < count:
        a, b = sorted(int(x) for x in rng.integers(0, N, 2))
        if b - a < max(1, N // 4) or (a, b) in seen:
            if N < 4:  # tiny grids: any distinct pair
                if a == b:
                    continue
            else:
                continue
        seen.add((a, b))
        frm.append(a)
        to.append(b)
    kind0 = np.zeros(L, np.int32) if inst.line_kind is None else np.asarray(inst.line_kind, np.int32)
    outage = np.asarray(inst.outage, np.int32).copy()
    if outage_first and int(inst.K) >= 1 and count >= 1:
        outage[0] = L
    return _dc.replace(
        inst,
        line_from=np.r_[inst.line_from, frm].astype(np.int32),
        line_to=np.r_[inst.line_to, to].astype(np.int32),
        line_sus=np.r_[inst.line_sus, np.full(count, 10.0)],
        line_cap=np.r_[inst.line_cap, rng.uniform(cap[0], cap[1], count)],
        outage=outage,
        line_kind=np.r_[kind0, np.ones(count, np.int32)],
    )


def with_contingency_changes(inst: Instance, seed: int = 0, second_outages: int = 2,
                             rating_changes: int = 6, sus_changes: int = 3) -> Instance:
    """The same network with general per-contingency line parameters (Section
    2.3: contingency k may change any line's parameters, not only remove one):

    * `second_outages` contingencies also lose a second line (N-2), chosen so
      that the grid stays connected;
    * `rating_changes` (contingency, line) pairs get a post-contingency
      (emergency) capacity U[1.1, 1.5] times the base one;
    * `sus_changes` pairs get a susceptance U[0.5, 0.9] times the base one
      (a switched series device) with the base capacity.

    Pairs are distinct and never the contingency's own N-1 outage."""
    import dataclasses as _dc
    rng = np.random.default_rng([seed, 0xC4])
    K, L, N = int(inst.K), len(inst.line_from), int(inst.N)
    frm, to = np.asarray(inst.line_from), np.asarray(inst.line_to)
    outage = np.asarray(inst.outage)
    used = {(k + 1, int(outage[k])) for k in range(K) if outage[k] >= 0}
    ks, ls, bs, us = [], [], [], []
    sus = np.asarray(inst.line_sus, float)
    cap = np.asarray(inst.line_cap, float)

    def free_pair(k):
        for _ in range(1000):
            l = int(rng.integers(0, L))
            if (k, l) not in used:
                return l
        raise RuntimeError("no free (contingency, line) pair")

    if K >= 1 and second_outages > 0:
        for k in rng.choice(np.arange(1, K + 1), min(second_outages, K), replace=False):
            k = int(k)
            for _ in range(1000):
                l = free_pair(k)
                keep = np.ones(L, bool)
                keep[l] = False
                if outage[k - 1] >= 0:
                    keep[outage[k - 1]] = False
                if len(np.unique(_components(N, np.stack([frm[keep], to[keep]], 1)))) == 1:
                    break
            else:
                raise RuntimeError("no second outage keeps the grid connected")
            used.add((k, l))
            ks.append(k); ls.append(l); bs.append(0.0); us.append(0.0)
    for n_pairs, kind in ((rating_changes, "cap"), (sus_changes, "sus")):
        for _ in range(n_pairs if K >= 1 else 0):
            k = int(rng.integers(1, K + 1))
            l = free_pair(k)
            used.add((k, l))
            ks.append(k); ls.append(l)
            if kind == "cap":
                bs.append(sus[l]); us.append(cap[l] * rng.uniform(1.1, 1.5))
            else:
                bs.append(sus[l] * rng.uniform(0.5, 0.9)); us.append(cap[l])
    return _dc.replace(inst, chg_k=np.asarray(ks, np.int32), chg_line=np.asarray(ls, np.int32),
                       chg_sus=np.asarray(bs, float), chg_cap=np.asarray(us, float))
