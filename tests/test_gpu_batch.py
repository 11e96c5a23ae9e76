"""Batched uneven instances: every phase is one launch over all instances.

Each instance of a batch must give the iterates it gives alone (and the
oracle's), keep its own penalty sequence and convergence, and the autotuner
must leave the iterate at the zero start.
"""
import functools
import math
import os
import sys
import tempfile

import numpy as np
import pytest
import torch

from oracle.mp import Options, Solver as Oracle
from paper_2410_17203_amd import synth
from tests.parity import BARS, FIELDS, compare_fields

pytestmark = pytest.mark.gpu

# a batch member against the same instance alone: the same kernels in the
# same summation order
SAME = dict(l2=1e-12, elem=1e-11, floor=1e-4)

SHAPES = [  # N, T, K: uneven horizon, contingency count and size
    (30, 1, 0), (80, 24, 5), (120, 24, 12), (60, 48, 30), (200, 1, 3), (20, 48, 7),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def batch_instances():
    out = []
    for i, (N, T, K) in enumerate(SHAPES):
        out.append(synth.make_instance(f"b{i}", N=N, L=int(round(1.4 * N)), G=max(2, N // 5),
                                       D=int(0.8 * N), B=max(1, N // 25), T=T, K=K,
                                       seed=900 + i))
    out[2] = synth.with_dc_links(out[2], 3, seed=2)  # DC links beside AC-only instances
    out[3] = synth.with_contingency_changes(out[3], seed=3)  # per-contingency changes
    return out


@functools.lru_cache(maxsize=None)
def oracle_state(i, iters):
    o = Oracle(batch_instances()[i], Options(adapt_every=0, eps=1e-12))
    o.run(iters)
    return o.canonical_state()


def rel_err(a, b):
    nb = float(torch.linalg.norm(b))
    na = float(torch.linalg.norm(a - b))
    return na if nb == 0.0 else na / nb


@pytest.mark.parametrize("tiles", [0, 1])
def test_batched_iterates_match_oracle_per_instance(tiles):
    """Batched node-row sweep (tiles = 0) and batched tiled sweep over all
    instances' tiles (tiles = 1)."""
    from paper_2410_17203_amd.binding import Solver
    say(f"[batch] fp64 vs oracle, tiles={tiles}")
    insts = batch_instances()
    s = Solver(insts, dtype="f64", adapt_every=0, eps=1e-12, sweep_tiles=tiles)
    assert s.num_instances == len(insts)
    s.iterate(150)
    for i in range(len(insts)):
        ref = oracle_state(i, 150)
        compare_fields(lambda f: s.field(f, i), ref, BARS["f64"])
        assert s.residuals(i)["iter"] == 150
    s.close()


@pytest.mark.parametrize("tiles", [0, 1])
def test_batched_equals_one_at_a_time(tiles):
    from paper_2410_17203_amd.binding import Solver
    say(f"[batch] batched vs single, adaptive penalty, tiles={tiles}")
    insts = batch_instances()
    b = Solver(insts, dtype="f64", eps=1e-12, rho_p=0.2, rho_theta=5.0, sweep_tiles=tiles)
    b.iterate(120)
    for i, inst in enumerate(insts):
        a = Solver(inst, dtype="f64", eps=1e-12, rho_p=0.2, rho_theta=5.0, sweep_tiles=tiles)
        a.iterate(120)
        ha, hb = a.history(), b.history(instance=i)
        assert [(h["rho_p"], h["rho_theta"]) for h in ha] == \
            [(h["rho_p"], h["rho_theta"]) for h in hb]
        compare_fields(lambda f: b.field(f, i), a.state(), SAME)
        a.close()
    b.close()


@pytest.mark.parametrize("tiles", [0, 1])
def test_batched_solve_stops_each_instance_on_its_own(tiles):
    from paper_2410_17203_amd.binding import Solver
    say(f"[batch] solve fp32, tiles={tiles}")
    insts = batch_instances()
    cap = 6000
    b = Solver(insts, dtype="f32", eps=1e-3, max_iter=cap, sweep_tiles=tiles)
    r = b.solve()
    res = [b.residuals(i) for i in range(len(insts))]
    conv = [x["converged"] for x in res]
    assert r["status"] == ("OPF_OK" if all(conv) else "OPF_NOT_CONVERGED")
    # the single-period instances converge early, at different iterations
    done = [x["iter"] for x in res if x["converged"]]
    assert len(done) >= 2 and len(set(done)) == len(done)
    for x in res:
        if x["converged"]:
            assert x["iter"] < cap
            assert max(x["rms_primal"], x["rms_dual"]) <= x["threshold"]
        else:
            assert x["iter"] == cap
    # stopped instances (converged or at the cap) stay where they stopped
    b.iterate(100)
    for i, x in enumerate(res):
        assert b.residuals(i)["iter"] == x["iter"]
    # the solve left stopped instances out of its work lists as they stopped;
    # the lists are whole again afterwards: a second solve from zero repeats
    # the first one bit for bit
    b.reset()
    b.solve()
    for i, x in enumerate(res):
        y = b.residuals(i)
        assert (y["iter"], y["converged"], y["objective"], y["rms_primal"], y["rms_dual"]) == \
            (x["iter"], x["converged"], x["objective"], x["rms_primal"], x["rms_dual"]), i
    # each instance stops where its own single-instance solve stops
    for i, inst in enumerate(insts):
        a = Solver(inst, dtype="f32", eps=1e-3, max_iter=cap, polish_fp64=0, sweep_tiles=tiles)
        ra = a.solve()
        assert ra["iter"] == res[i]["iter"] and ra["converged"] == res[i]["converged"]
        assert abs(ra["objective"] - res[i]["objective"]) <= 1e-5 * abs(ra["objective"])
        a.close()
    b.close()


def test_autotune_resets_and_caches():
    from paper_2410_17203_amd.binding import Solver
    say("[batch] autotune")
    insts = batch_instances()
    b = Solver(insts, dtype="f64", adapt_every=0, eps=1e-12)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        t1 = b.autotune(trials=3, cache_path=path)
        assert t1["from_cache"] == 0 and t1["ms_per_iter"] > 0
        assert t1["lanes_shift"] in (-1, 0, 1) and t1["grid_factor"] in (0.5, 1.0, 2.0)
        t2 = b.autotune(trials=3, cache_path=path)
        assert t2["from_cache"] == 1 and t2["lanes_shift"] == t1["lanes_shift"]
    assert b.residuals(0)["iter"] == 0  # back at the zero start
    b.iterate(150)
    for i in [1, 3]:
        compare_fields(lambda f: b.field(f, i), oracle_state(i, 150), BARS["f64"])
    b.close()


def test_autotune_times_full_iterations_whatever_the_stopping_options():
    """Trial iterations ignore max_iter and the tolerance (an instance that
    stopped would make later trials no-ops and win them), and the options
    are back in force afterwards."""
    from paper_2410_17203_amd.binding import Solver
    say("[batch] autotune under tight stopping options")
    insts = batch_instances()
    free = Solver(insts, dtype="f32", eps=0.0, max_iter=10**6)
    t_free = free.autotune(trials=8)
    free.close()
    tight = Solver(insts, dtype="f32", eps=1e-1, max_iter=2)
    t_tight = tight.autotune(trials=8)
    say(f"  ms/iteration: {t_free['ms_per_iter']:.4f} free, {t_tight['ms_per_iter']:.4f} tight")
    assert t_tight["ms_per_iter"] > 0.5 * t_free["ms_per_iter"]
    tight.solve()
    # max_iter is back in force after the trials
    assert max(tight.residuals(i)["iter"] for i in range(len(insts))) == 2
    tight.close()


def test_batched_bf16_duals_run():
    from paper_2410_17203_amd.binding import Solver
    say("[batch] bf16 duals")
    insts = batch_instances()
    b = Solver(insts, dtype="f32", dual_dtype="bf16", adapt_every=0, eps=1e-12)
    b.iterate(150)
    for i in range(len(insts)):
        r = b.residuals(i)
        assert math.isfinite(r["rms_primal"]) and math.isfinite(r["rms_dual"])
    err = rel_err(b.field("P", 2), oracle_state(2, 150)["P"])
    say(f"  bf16 relative error of P (instance 2) vs oracle: {err:.2e}")
    assert err < 5e-2
    b.close()


def _mixed_batch():
    """Large multi-period instances with small single-period instances
    between them: with more tiles than workgroups, a workgroup's stride
    through its XCD's range of tiles steps over whole small instances."""
    out = []
    for i in range(12):
        if i % 2 == 0:
            out.append(synth.make_instance(f"m{i}", N=300, L=420, G=60, D=240, B=12, T=24, K=4,
                                           seed=700 + i))
        else:
            out.append(synth.make_instance(f"m{i}", N=40, L=56, G=8, D=32, B=2, T=1, K=2,
                                           seed=700 + i))
    return out


def _tuning_cache(path, insts, precision, grid_factor):
    """A cache line of opf_autotune for this batch (key: device, precision,
    batch shape) that selects the given sweep grid factor."""
    arch = torch.cuda.get_device_properties(0).gcnArchName
    sN = sum(x.N * x.T for x in insts)
    sL = sum(x.L * x.T for x in insts)
    sKT = sum((x.K + 1) * x.T for x in insts)
    key = f"{arch}|p{precision}|n{len(insts)}|NT{sN}|LT{sL}|KT{sKT}"
    with open(path, "w") as fh:
        fh.write(f"{key} 0 {grid_factor} -1 1 1.0\n")


def test_batch_residuals_survive_a_smaller_grid():
    """Regression: after a run with a large tiled-sweep grid, a run with a
    smaller one (the autotuner switching configurations) must not sum
    residual partials left behind by the first run.  Every instance's
    residual record and penalty sequence equal its own single-instance run."""
    from paper_2410_17203_amd.binding import Solver
    say("[batch] residual partials across grid sizes")
    insts = _mixed_batch()
    b = Solver(insts, dtype="f64", eps=1e-12, rho_p=0.3, rho_theta=3.0)
    with tempfile.TemporaryDirectory() as d:
        big, small = os.path.join(d, "big.txt"), os.path.join(d, "small.txt")
        _tuning_cache(big, insts, 0, 2.0)
        _tuning_cache(small, insts, 0, 0.5)
        t = b.autotune(trials=1, cache_path=big)
        assert t["from_cache"] == 1 and t["grid_factor"] == 2.0
        b.iterate(30)
        b.synchronize()
        t = b.autotune(trials=1, cache_path=small)
        assert t["from_cache"] == 1 and t["grid_factor"] == 0.5
    b.iterate(60)
    for i, inst in enumerate(insts):
        a = Solver(inst, dtype="f64", eps=1e-12, rho_p=0.3, rho_theta=3.0)
        a.iterate(60)
        ha, hb = a.history(), b.history(instance=i)
        assert len(ha) == len(hb) == 60
        for x, y in zip(ha, hb):
            assert (x["rho_p"], x["rho_theta"]) == (y["rho_p"], y["rho_theta"]), i
            # the partial sums differ in order from the single-instance
            # sweep's: agreement to rounding (the expanded dual power norm
            # cancels, so it is held against the primal norm's size)
            for key in ("primal_p", "primal_theta", "dual_p", "dual_theta"):
                den = max(abs(x[key]), 1e-6 * x["primal_p"], 1e-300)
                assert abs(x[key] - y[key]) <= 1e-7 * den, (i, x["iter"], key, x[key], y[key])
        a.close()
    b.close()
