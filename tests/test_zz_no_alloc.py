"""opf_load_network_static (the fixed per-device workspace, for callers that
cannot allocate device memory) against opf_load_network with a caller
workspace: the same instance gives the same iterate, residual record and
solve, on two loads in a row, the second with a smaller network; networks
beyond the fixed size are rejected; a second context taking the array over
leaves the first unloaded."""
import sys

import numpy as np
import pytest
import torch

from paper_2410_17203_amd import synth
from tests.parity import FIELDS

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(a, b, iters):
    a.iterate(iters)
    b.iterate(iters)
    for f in FIELDS:
        assert torch.equal(a.field(f), b.field(f)), f
    assert a.history() == b.history()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_static_workspace_matches_caller_workspace(dtype):
    from paper_2410_17203_amd.binding import Solver
    big = synth.config("diff")                      # 39 MiB FP64 workspace
    small = synth.config("tiny", T=6, K=3, seed=4, B=2)
    opts = dict(dtype=dtype, polish_fp64=0, rho_p=0.4, rho_theta=2.0)
    s = Solver(big, static_workspace=True, **opts)
    assert s.workspace_bytes <= 64 << 20
    say(f"[static] {dtype} first load: {s.workspace_bytes / 2**20:.1f} MiB")
    ref = Solver(big, **opts)
    _same(s, ref, 120)
    ref.close()
    # second call on the same context, smaller network: what the first load
    # left in the array must not leak into it
    s.load(small, static_workspace=True)
    say("[static] second load, smaller network")
    ref = Solver(small, **opts)
    _same(s, ref, 150)
    rs = s.solve()
    rr = ref.solve()
    assert (rs["iter"], rs["objective"], rs["status"]) == (rr["iter"], rr["objective"], rr["status"])
    ref.close()
    s.close()


def test_static_workspace_limits_and_takeover():
    from paper_2410_17203_amd.binding import OpfError, Solver
    with pytest.raises(OpfError, match="OPF_E_OOM.*fixed workspace holds 67108864"):
        Solver(synth.config("medium"), dtype="f64", static_workspace=True)
    a = Solver(synth.config("tiny"), dtype="f64", static_workspace=True)
    a.iterate(5)
    b = Solver(synth.config("tiny", K=2), dtype="f64", static_workspace=True)
    with pytest.raises(OpfError, match="took over"):
        a.iterate(5)
    b.iterate(5)
    assert b.residuals()["iter"] == 5
    a.close()
    b.close()
