"""Comparison of a field of the HIP iterate with the oracle's, used by the
GPU parity tests.

Two measures per field, both required:

* the relative L2 error ||g - r|| / ||r|| (the parity bar: 1e-10 for the
  FP64 iterate, 1e-4 for FP32, after 200 iterations);
* the largest elementwise error |g - r| / (|r| + floor S), so that a
  single wrong element (a wrong ragged tail, one bad contingency slot)
  cannot hide inside a norm over 10^5..10^6 elements.  S is the field's
  largest magnitude, or for an average of other quantities the largest
  magnitude of what it averages (pbar averages the terminal powers, whose
  rounding it inherits, and is small where the network nearly balances;
  the device phase duals VNC average the contingencies' duals).  The floor
  keeps elements that are zero to rounding from dominating: below floor S
  an element is held to an absolute bound.  FP64: tolerance 1e-9 at floor
  1e-4.  FP32: 5e-3 at floor 1e-2; the FP32 unit roundoff is 6e-8, the
  200-iteration L2 errors are 1e-7..1e-4 and the measured elementwise
  errors up to about 1e-3 (the iteration amplifies rounding near clip
  boundaries), so this bound still fails any element off by more than half
  a percent of its magnitude or of 1% of the field's scale.
"""
import torch

FIELDS = ["P", "TH1", "TH2", "V1", "V2", "U", "PBAR", "THBAR", "PNC", "THNC", "VNC"]

BARS = {"f64": dict(l2=1e-10, elem=1e-9, floor=1e-4),
        "f32": dict(l2=1e-4, elem=5e-3, floor=1e-2)}

# fields that average other fields: their elementwise scale includes what
# they average
SUMMANDS = {"PBAR": ("P", "PNC"), "VNC": ("V1", "V2")}


def rel_l2(g, r):
    nr = float(torch.linalg.norm(r))
    ne = float(torch.linalg.norm(g - r))
    return ne if nr == 0.0 else ne / nr


def rel_elem(g, r, floor, scale=0.0):
    if r.numel() == 0:
        return 0.0
    big = max(float(r.abs().max()), scale)
    if big == 0.0:
        return float((g - r).abs().max())
    return float(((g - r).abs() / (r.abs() + floor * big)).max())


def compare_fields(get, ref, bar, fields=FIELDS, skip=()):
    """get(name) -> FP64 CPU tensor of the HIP iterate; ref: the oracle's
    canonical state; bar: a BARS entry (or a dict with l2, elem, floor).
    Returns {field: (l2, elem)}; fails listing every field beyond its bar."""
    out, bad = {}, {}
    for f in fields:
        if f in skip:
            continue
        g = get(f)
        r = ref[f].to(torch.float64)
        assert g.shape == r.shape, (f, tuple(g.shape), tuple(r.shape))
        scale = max([float(ref[q].abs().max()) for q in SUMMANDS.get(f, ()) if ref[q].numel()],
                    default=0.0)
        l2, el = rel_l2(g, r), rel_elem(g, r, bar["floor"], scale)
        out[f] = (l2, el)
        if not (l2 <= bar["l2"] and el <= bar["elem"]):
            bad[f] = (l2, el)
    assert not bad, f"fields beyond (l2 {bar['l2']}, elem {bar['elem']}): {bad}; all: {out}"
    return out
