"""The iterate through the ABI: zero-copy layout views, export and import
(warm start, Section 3.4)."""
import sys

import numpy as np
import pytest
import torch

from paper_2410_17203_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small(seed=21, **kw):
    args = dict(N=40, L=56, G=8, D=30, B=3, T=12, K=37, seed=seed)  # two chunks
    args.update(kw)
    return synth.make_instance("state", **args)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_layout_views_match_exported_fields(dtype):
    from paper_2410_17203_amd.binding import Solver
    say(f"[state] layout views {dtype}")
    inst = small()
    s = Solver(inst, dtype=dtype, polish_fp64=0)
    s.iterate(23)
    Kp = inst.K + 1
    P = s.field("P")                                         # [K+1, L, T]
    v = torch.cat(s.view("P"), dim=2).double().cpu()          # [T, L, Kpp]
    assert torch.equal(v[:, :, :Kp].permute(2, 1, 0), P)
    U = s.field("U")
    u = torch.cat(s.view("U"), dim=2).double().cpu()
    assert torch.equal(u[:, :, :Kp].permute(2, 1, 0), U)
    assert torch.equal(s.view("pnc").double().cpu(), s.field("PNC"))
    s.close()


@pytest.mark.parametrize("split", [50, 47])
def test_export_import_continues_bitwise(split):
    """Stopping after `split` iterations (50: right after a penalty change is
    decided, with a rescale still pending), exporting, importing into a new
    context and running on gives the same iterates as running straight on."""
    from paper_2410_17203_amd.binding import Solver
    say(f"[state] export/import at {split}")
    inst = small()
    opts = dict(rho_p=0.2, rho_theta=4.0, polish_fp64=0)
    a = Solver(inst, dtype="f64", **opts)
    a.iterate(split)
    blob = a.get_state()
    a.iterate(40)
    b = Solver(inst, dtype="f64", **opts)
    if split % 10 == 0:
        b.set_state(blob)
        b.iterate(40)
        for f in ["P", "TH1", "V2", "U", "THBAR", "PNC", "VNC"]:
            assert torch.equal(a.field(f), b.field(f)), f
        assert b.residuals()["rho_p"] == a.residuals()["rho_p"]
    else:
        # off the penalty-update phase the adaptive schedule shifts; with the
        # rule off the continuation is still exact
        c = Solver(inst, dtype="f64", adapt_every=0, **opts)
        c.iterate(split)
        blob0 = c.get_state()
        c.iterate(40)
        d = Solver(inst, dtype="f64", adapt_every=0, **opts)
        d.set_state(blob0)
        d.iterate(40)
        for f in ["P", "TH1", "V2", "U", "THBAR", "PNC", "VNC"]:
            assert torch.equal(c.field(f), d.field(f)), f
        c.close()
        d.close()
    a.close()
    b.close()


def test_warm_start_takes_fewer_iterations():
    """Solve, perturb the loads by a few percent (the next day's forecast),
    solve again from the previous iterate: fewer iterations than from zero,
    at a tolerance of 1e-4.  The grid's two outages are lines that a
    redispatch idles, so the problem is feasible with the device phases
    shared by all contingencies (Section 2.3; the oracle reaches 1e-4 in
    2,377 iterations).  Two solves stopped at that relative tolerance agree
    in objective to 1e-3; tests/test_gpu_warm.py checks the same warm and
    cold solves against the oracle to 1e-9."""
    from paper_2410_17203_amd.binding import Solver
    say("[state] warm start")
    shape = dict(synth.CONFIGS["tiny"])
    shape["K"] = 2
    inst = synth.make_instance("state", **shape)
    s = Solver(inst, dtype="f64", eps=1e-4, max_iter=30000)
    r0 = s.solve()
    assert r0["status"] == "OPF_OK"
    blob = s.get_state()
    s.close()
    nxt = synth.make_instance("state", **shape)
    rng = np.random.default_rng(1)
    nxt.load_d = np.asarray(inst.load_d) * (1.0 + 0.03 * rng.standard_normal(np.shape(inst.load_d)))
    cold = Solver(nxt, dtype="f64", eps=1e-4, max_iter=30000)
    rc = cold.solve()
    warm = Solver(nxt, dtype="f64", eps=1e-4, max_iter=30000)
    warm.set_state(blob)
    rw = warm.solve()
    say(f"  cold {rc['iter']} iterations, warm {rw['iter']} (day 1: {r0['iter']})")
    assert rc["status"] == rw["status"] == "OPF_OK"
    assert rw["iter"] < rc["iter"]
    # both stop at the same residual tolerance; their objectives agree to its order
    assert abs(rw["objective"] - rc["objective"]) <= 1e-3 * abs(rc["objective"])
    cold.close()
    warm.close()


def test_import_rejects_mismatched_state():
    from paper_2410_17203_amd.binding import OpfError, Solver
    say("[state] rejects")
    a = Solver(small(), dtype="f64")
    a.iterate(3)
    blob = a.get_state()
    b = Solver(small(K=4), dtype="f64")
    with pytest.raises(OpfError, match="another shape"):
        b.set_state(blob)
    bad = blob.clone()
    bad[:8] = 0
    with pytest.raises(OpfError, match="not a state"):
        a.set_state(bad)
    # same sizes, different wiring: two lines swap their to nodes
    other = small()
    lt = np.asarray(other.line_to).copy()
    i, j = next((i, j) for i in range(len(lt)) for j in range(i + 1, len(lt))
                if lt[i] != lt[j] and other.line_from[i] != lt[j] and other.line_from[j] != lt[i])
    lt[i], lt[j] = lt[j], lt[i]
    other.line_to = lt
    c = Solver(other, dtype="f64")
    with pytest.raises(OpfError, match="another structure"):
        c.set_state(blob)
    # different loads on the same structure are accepted (a warm start)
    day2 = small()
    day2.load_d = np.asarray(day2.load_d) * 1.01
    d = Solver(day2, dtype="f64")
    d.set_state(blob)
    for x in (a, b, c, d):
        x.close()


def test_dc_link_state_view_and_continuation():
    """With DC links the iterate holds their half phase differences (view
    'Hd', equal to (TH1 - TH2)/2 of each link in every contingency), and an
    exported state carries them: the continuation is bitwise identical."""
    from paper_2410_17203_amd.binding import Solver
    say("[state] DC links")
    inst = synth.with_dc_links(small(), 3, seed=9)
    dcl = np.nonzero(inst.line_kind == 1)[0]
    opts = dict(adapt_every=0, polish_fp64=0)
    a = Solver(inst, dtype="f64", **opts)
    a.iterate(30)
    lay = a.layout()
    assert lay["Ldc"] == 3
    hd = torch.cat(a.view("Hd"), dim=2).double().cpu()[:, :, :inst.K + 1]   # [T, Ldc, K+1]
    half = 0.5 * (a.field("TH1") - a.field("TH2"))[:, dcl, :]                # [K+1, Ldc, T]
    # TH1, TH2 = Tm +- Hd, so (TH1 - TH2)/2 recovers Hd up to the rounding of Tm +- Hd
    torch.testing.assert_close(hd.permute(2, 1, 0), half, rtol=0, atol=1e-15)
    assert float(half.abs().max()) > 0
    blob = a.get_state()
    a.iterate(25)
    b = Solver(inst, dtype="f64", **opts)
    b.set_state(blob)
    b.iterate(25)
    for f in ["P", "TH1", "TH2", "V1", "U", "THBAR", "PNC"]:
        assert torch.equal(a.field(f), b.field(f)), f
    c = Solver(synth.with_dc_links(small(), 2, seed=9), dtype="f64", **opts)
    with pytest.raises(Exception, match="another shape"):
        c.set_state(blob)
    for x in (a, b, c):
        x.close()


def test_change_state_view_and_continuation():
    """With lines taken out by per-contingency changes the iterate holds their
    half phase differences (view 'Tz', in the order of the change list), and
    an exported state carries them."""
    from paper_2410_17203_amd.binding import Solver
    say("[state] per-contingency changes")
    inst = synth.with_contingency_changes(small(), seed=3, second_outages=3, rating_changes=5,
                                          sus_changes=4)
    out = inst.chg_sus == 0
    opts = dict(adapt_every=0, polish_fp64=0)
    a = Solver(inst, dtype="f64", **opts)
    a.iterate(30)
    lay = a.layout()
    assert lay["Zc"] == int(out.sum()) == 3
    tz = a.view("Tz").double().cpu()                                   # [T, Zc]
    th1, th2 = a.field("TH1"), a.field("TH2")                          # [K+1, L, T]
    k, l = inst.chg_k[out], inst.chg_line[out]
    half = 0.5 * (th1 - th2)[k, l, :]                                  # [Zc, T]
    torch.testing.assert_close(tz.T, half, rtol=0, atol=1e-15)
    assert float(half.abs().max()) > 0
    assert torch.all(a.field("P")[k, l, :] == 0)
    blob = a.get_state()
    a.iterate(25)
    b = Solver(inst, dtype="f64", **opts)
    b.set_state(blob)
    b.iterate(25)
    for f in ["P", "TH1", "TH2", "V1", "U", "THBAR", "PNC"]:
        assert torch.equal(a.field(f), b.field(f)), f
    c = Solver(small(), dtype="f64", **opts)
    with pytest.raises(Exception, match="another shape"):
        c.set_state(blob)
    for x in (a, b, c):
        x.close()
