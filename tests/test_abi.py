"""The C-ABI library loads, exports every declared symbol, and its host-side
validation and sizing logic behaves as documented (no device work)."""
import ctypes

import numpy as np
import pytest

from paper_2410_17203_amd import binding, synth


@pytest.fixture(scope="module")
def lib():
    return binding.load_library()


def test_exports_every_declared_symbol(lib):
    names = binding.header_functions()
    assert len(names) >= 15
    for n in ["opf_create", "opf_load_network", "opf_iterate", "opf_solve", "opf_residuals"]:
        assert n in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing


def test_default_options_follow_the_paper(lib):
    o = binding.default_options()
    # Section 5.2: rho = 1, mu = 2, gamma = 1.1 every 10 iterations; Section
    # 4.5: 10 inner iterations
    assert (o.rho_p, o.rho_theta, o.mu, o.gamma, o.adapt_every) == (1.0, 1.0, 2.0, 1.1, 10)
    assert o.inner_iters == 10 and o.check_every == 1 and o.block_iters == 50
    assert o.polish_fp64 == 1 and o.polish_factor == 1.2
    assert o.sweep_tiles == -1


def _ctx(lib, **kw):
    o = binding.default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    st = lib.opf_create(ctypes.byref(o), ctypes.byref(ctx))
    return st, ctx


def _wsize(lib, ctx, inst):
    arr = binding.NetworkArrays(inst)
    n = ctypes.c_size_t()
    st = lib.opf_workspace_size(ctx, ctypes.byref(arr.net), ctypes.byref(n))
    return st, n.value, lib.opf_last_error(ctx).decode()


def test_option_validation(lib):
    assert _ctx(lib, rho_p=0.0)[0] == -1
    assert _ctx(lib, adapt_every=10, check_every=3)[0] == -1
    assert _ctx(lib, state_dtype=binding.F64, dual_dtype=binding.BF16)[0] == -1
    assert _ctx(lib, inner_iters=0)[0] == -1
    assert _ctx(lib, polish_factor=0.5)[0] == -1
    assert _ctx(lib, sweep_tiles=2)[0] == -1
    st, ctx = _ctx(lib, state_dtype=binding.F32, dual_dtype=binding.BF16)
    assert st == 0
    lib.opf_destroy(ctx)


def test_workspace_size_scales_with_contingencies(lib):
    st, ctx = _ctx(lib)
    assert st == 0
    small = synth.config("tiny", T=4, K=2, seed=3)
    big = synth.config("tiny", T=4, K=9, seed=3)
    s1, n1, _ = _wsize(lib, ctx, small)
    s2, n2, _ = _wsize(lib, ctx, big)
    assert s1 == 0 and s2 == 0 and n2 > n1 > 0
    lib.opf_destroy(ctx)


@pytest.mark.parametrize("mutate,needle", [
    (lambda i: i.line_sus.__setitem__(0, 0.0), "susceptance"),
    (lambda i: i.line_cap.__setitem__(1, -1.0), "capacity"),
    (lambda i: i.line_from.__setitem__(2, 99), "out of range"),
    (lambda i: i.gen_c2.__setitem__(0, -1e-3), "c2 >= 0"),
    (lambda i: i.gen_pmax.__setitem__((0, 0), -5.0), "pmin <= pmax"),
    (lambda i: i.load_d.__setitem__((0, 0), np.nan), "load demand"),
    (lambda i: i.bat_eta.__setitem__(0, 1.5), "eta"),
    (lambda i: setattr(i, "outage", np.array([3, 3], np.int32)), "distinct"),
])
def test_invalid_networks_are_rejected(lib, mutate, needle):
    st, ctx = _ctx(lib)
    inst = synth.config("tiny", T=2, K=2, B=2, seed=11)
    mutate(inst)
    s, _, msg = _wsize(lib, ctx, inst)
    assert s == -1 and needle in msg
    lib.opf_destroy(ctx)


def test_isolated_node_rejected(lib):
    st, ctx = _ctx(lib)
    inst = synth.two_node()
    inst.N = 3  # node 2 has no terminal
    s, _, msg = _wsize(lib, ctx, inst)
    assert s == -1 and "no terminal" in msg
    lib.opf_destroy(ctx)


def test_contingency_limit_per_precision(lib):
    inst = synth.config("tiny", K=0)
    inst.K = 600
    inst.outage = -np.ones(600, np.int32)
    st, ctx = _ctx(lib)  # FP64 iterate: K+1 <= 512
    s, _, msg = _wsize(lib, ctx, inst)
    assert s == -1 and "K too large" in msg
    lib.opf_destroy(ctx)
    st, ctx = _ctx(lib, state_dtype=binding.F32, dual_dtype=binding.F32, polish_fp64=0)
    s, _, _ = _wsize(lib, ctx, inst)
    assert s == 0
    lib.opf_destroy(ctx)


def test_calls_before_load_are_state_errors(lib):
    st, ctx = _ctx(lib)
    assert lib.opf_iterate(ctx, 1) == -4
    r = binding.Resid()
    assert lib.opf_residuals(ctx, ctypes.byref(r)) == -4
    lib.opf_destroy(ctx)


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (compiled from include/opf.h with the host C compiler)."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"opf_options": binding.Options, "opf_network": binding.Network,
               "opf_resid": binding.Resid, "opf_tuning": binding.Tuning,
               "opf_layout": binding.Layout}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "opf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
