"""Degenerate and maximum-size inputs against the oracle: the largest
contingency count the library accepts (several chunks of contingencies in a
single line row), a network without lines, and a single node with a
generator, a load and a battery."""
import sys

import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver as Oracle
from paper_2410_17203_amd import synth
from tests.parity import BARS, FIELDS, compare_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    nb = float(torch.linalg.norm(b))
    na = float(torch.linalg.norm(a - b))
    return na if nb == 0.0 else na / nb


def max_k(K):
    """The 14-node grid with K contingencies: every non-bridge line outaged
    once, the rest no-op contingencies."""
    inst = synth.config("tiny")
    is_bridge = synth.bridges(inst.N, np.asarray(inst.line_from), np.asarray(inst.line_to))
    cand = np.nonzero(~is_bridge)[0]
    out = -np.ones(K, np.int32)
    out[:len(cand)] = cand
    inst.K = K
    inst.outage = out
    return inst


def isolated(N=3, T=4, B=1, seed=0):
    """N nodes with no lines, each with a generator and a load (node 0 also
    with a battery): N independent single-node dispatch problems."""
    rng = np.random.default_rng(seed)
    f = lambda v: np.asarray(v, np.float64)
    return synth.Instance(
        name="isolated", N=N, T=T, K=0,
        line_from=np.zeros(0, np.int32), line_to=np.zeros(0, np.int32),
        line_sus=f([]), line_cap=f([]), outage=np.zeros(0, np.int32),
        gen_node=np.arange(N, dtype=np.int32), gen_c2=rng.uniform(0.01, 0.1, N),
        gen_c1=rng.uniform(10, 50, N), gen_pmin=np.zeros((N, T)), gen_pmax=np.full((N, T), 3.0),
        gen_ramp=np.full(N, 0.5),
        load_node=np.arange(N, dtype=np.int32), load_d=rng.uniform(0.5, 1.5, (N, T)),
        bat_node=np.zeros(B, np.int32), bat_P=f([0.5] * B), bat_dur=f([4.0] * B),
        bat_eta=f([0.9] * B), bat_alpha=f([1.0] * B), meta={})


CASES = [
    ("max_k_f32", lambda: max_k(1023), "f32"),
    ("max_k_f64", lambda: max_k(511), "f64"),
    ("no_lines", lambda: isolated(N=3), "f64"),
    ("single_node", lambda: isolated(N=1, T=24), "f64"),
]


@pytest.mark.parametrize("tiles", [0, 1])
@pytest.mark.parametrize("name,builder,dtype", CASES, ids=[c[0] for c in CASES])
def test_edge_case_iterates_match_oracle(name, builder, dtype, tiles):
    from paper_2410_17203_amd.binding import Solver
    say(f"[edge] {name} {dtype} tiles={tiles}")
    inst = builder()
    o = Oracle(inst, Options(adapt_every=0, eps=1e-12))
    o.run(150)
    ref = o.canonical_state()
    s = Solver(inst, dtype=dtype, adapt_every=0, eps=1e-12, polish_fp64=0, sweep_tiles=tiles)
    s.iterate(150)
    compare_fields(s.field, ref, BARS[dtype])
    r = s.residuals()
    assert r["iter"] == 150 and np.isfinite(r["rms_primal"])
    s.close()


def test_contingency_count_above_the_limit_is_rejected():
    from paper_2410_17203_amd.binding import OpfError, Solver
    with pytest.raises(OpfError, match="K too large"):
        Solver(max_k(1024), dtype="f32", polish_fp64=0)
    with pytest.raises(OpfError, match="K too large"):
        Solver(max_k(512), dtype="f64")


def test_dc_link_rules_are_enforced():
    """Line kinds other than 0/1 are rejected; a DC link's susceptance is
    ignored (any value, even 0, gives the same iterate)."""
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import OpfError, Solver
    base = synth.make_instance("dc_rules", N=12, L=17, G=4, D=8, B=1, T=4, K=3, seed=5)
    inst = synth.with_dc_links(base, 2, seed=1)
    bad = inst.copy()
    bad.line_kind = bad.line_kind.copy()
    bad.line_kind[0] = 2
    with pytest.raises(OpfError, match="line kind"):
        Solver(bad, dtype="f64")
    s = Solver(inst, dtype="f64", polish_fp64=0)
    s.iterate(20)
    other = inst.copy()
    other.line_sus = np.asarray(other.line_sus, float).copy()
    other.line_sus[inst.line_kind == 1] = 0.0
    t = Solver(other, dtype="f64", polish_fp64=0)
    t.iterate(20)
    for f in ["P", "TH1", "TH2", "U"]:
        assert torch.equal(s.field(f), t.field(f)), f
    s.close()
    t.close()


def test_change_rules_are_enforced():
    """Invalid per-contingency changes are rejected (contingency or line out
    of range, a pair given twice, a pair repeating its contingency's outage,
    negative values)."""
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import OpfError, Solver
    base = synth.make_instance("chg_rules", N=12, L=17, G=4, D=8, B=1, T=4, K=3, seed=5)

    def with_chg(k, l, b, u):
        x = base.copy()
        x.chg_k, x.chg_line = np.array(k, np.int32), np.array(l, np.int32)
        x.chg_sus, x.chg_cap = np.array(b, float), np.array(u, float)
        return x

    free = [q for q in range(base.L) if q not in set(base.outage.tolist())]
    bad = [(with_chg([0], [free[0]], [1.0], [1.0]), "contingency out of range"),
           (with_chg([4], [free[0]], [1.0], [1.0]), "contingency out of range"),
           (with_chg([1], [base.L], [1.0], [1.0]), "line index out of range"),
           (with_chg([1, 1], [free[0], free[0]], [1.0, 2.0], [1.0, 1.0]), "changed twice"),
           (with_chg([2], [int(base.outage[1])], [1.0], [1.0]), "repeats its contingency"),
           (with_chg([1], [free[0]], [-1.0], [1.0]), "finite sus"),
           (with_chg([1], [free[0]], [1.0], [np.nan]), "finite sus")]
    for inst, msg in bad:
        with pytest.raises(OpfError, match=msg):
            Solver(inst, dtype="f64")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_infeasible_instance_stops_unconverged_with_finite_residuals(dtype):
    """Section 3.3: the iteration converges when the problem has a feasible
    point.  With the generators' total capacity at a fifth of the load there
    is none: opf_solve stops at max_iter with OPF_NOT_CONVERGED, the
    residuals stay finite and the primal residual stays above the tolerance,
    as in the oracle."""
    from paper_2410_17203_amd.binding import Solver
    say(f"[failure] infeasible {dtype}")
    inst = synth.config("tiny")
    inst.gen_pmax = np.asarray(inst.gen_pmax) * 0.2
    assert inst.gen_pmax[:, 0].sum() < 0.5 * inst.load_d[:, 0].sum()
    o = Oracle(inst, Options(eps=1e-3, max_iter=1500))
    ro = o.solve()
    assert not ro.converged and ro.iter == 1500
    s = Solver(inst, dtype=dtype, eps=1e-3, max_iter=1500)
    r = s.solve()
    assert r["status"] == "OPF_NOT_CONVERGED" and r["iter"] == 1500 and not r["converged"]
    assert np.isfinite(r["rms_primal"]) and np.isfinite(r["rms_dual"])
    assert r["rms_primal"] > r["threshold"]
    assert abs(r["rms_primal"] - ro.rms_primal) <= 1e-2 * ro.rms_primal
    for f in ["P", "U", "PNC"]:
        assert torch.isfinite(s.field(f)).all(), f
    s.close()


@pytest.mark.parametrize("dtype,demand", [("f32", 1e39), ("f64", 1e300)])
def test_overflow_is_reported_as_numeric_failure(dtype, demand):
    """A demand that is finite in FP64 but overflows the iterate (FP32) or
    the squared residual norms (FP64): the residual becomes infinite or NaN,
    the device stops iterating, and opf_solve and opf_residuals return
    OPF_E_NUMERIC rather than a converged or unconverged status."""
    from paper_2410_17203_amd.binding import OpfError, Solver
    say(f"[failure] overflow {dtype}")
    inst = synth.config("tiny")
    inst.load_d = np.asarray(inst.load_d).copy()
    inst.load_d[0, :] = demand
    s = Solver(inst, dtype=dtype, eps=1e-3, max_iter=500, polish_fp64=0)
    with pytest.raises(OpfError, match="OPF_E_NUMERIC"):
        s.solve()
    with pytest.raises(OpfError, match="OPF_E_NUMERIC"):
        s.residuals()
    # the device stopped at the first bad iteration
    s.iterate(20)
    h = s.history()
    assert len(h) <= 2
    s.close()
