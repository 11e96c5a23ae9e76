"""Code generation of the HIP kernels (host only: hipcc cross-compiles gfx950).

The batch kernels read each instance's descriptor from a table in device
memory.  Pointers loaded from that table must be known to address global
memory, or every access to the instance's state becomes a flat access; on
CDNA a flat access also counts against the LDS wait counter, so every LDS
barrier of the tiled sweep would wait for all HBM loads in flight (measured:
the 64-instance batch sweep 0.47 ms with global accesses, 0.65 ms with flat
ones).  This test compiles the kernels to gfx950 assembly with the library's
flags and checks that no kernel uses a flat memory instruction.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

from paper_2410_17203_amd import build


def _kernel_bodies(asm: str):
    """(symbol, instruction mnemonics) of every kernel in the assembly."""
    lines = asm.split("\n")
    starts = [(i, m.group(1)) for i, l in enumerate(lines)
              if (m := re.match(r"^(_Z\S*):", l))]
    for n, (i, name) in enumerate(starts):
        j = starts[n + 1][0] if n + 1 < len(starts) else len(lines)
        ops = []
        for l in lines[i + 1:j]:
            t = l.strip()
            if not t or t.startswith((";", ".")) or t.endswith(":"):
                continue
            ops.append(t.split()[0])
        yield name, ops


def test_no_kernel_uses_flat_memory_instructions(tmp_path):
    hipcc = build.hipcc()
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    flags = [f for f in build.HIP_FLAGS if f not in ("-shared", "-fPIC")]
    out = tmp_path / "opf_kernels.s"
    cmd = [hipcc, *flags, "-I", os.path.join(build.HERE, "..", "include"), "--cuda-device-only",
           "-S", os.path.join(build.CSRC, "opf_kernels.hip"), "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    kernels = dict(_kernel_bodies(out.read_text()))
    batch = [k for k in kernels if "_batch" in k]
    assert len(batch) >= 10, sorted(kernels)  # devices, sweeps, finalize, rescale per precision
    flat = {k: sum(op.startswith("flat_") for op in ops) for k, ops in kernels.items()}
    assert {k: v for k, v in flat.items() if v} == {}
    # the batch kernels do reach the state through global memory instructions
    for k in batch:
        assert any(op.startswith("global_") for op in kernels[k]), k
