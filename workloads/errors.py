"""Error measure used to compare recorded traces (no method arithmetic here).

The relative max-norm over recorded traces: for every record r,

    err_r = max |got_r - ref_r|  /  scale(class of r),

where the scale of a class is the max-norm of the reference over all
records of that class in the problem: the electric field (together with what
drives it: the source amplitudes and the max-norm of the initial field, e.g.
the random field that starts a laser), the magnetic field (the same divided by
the vacuum impedance), or density-matrix quantities (populations, inversions
and coherences).  A trace that stays near zero (an empty level, a field before
the pulse arrives, the field at a partly transparent facet) is thus measured
on the scale of its class, not on its own.
"""
from __future__ import annotations

import math

import numpy as np

_CLASS = {"e": "e", "h": "h", "pop": "rho", "inv": "rho", "rho_re": "rho", "rho_im": "rho"}


def class_scales(prob, ref):
    eta = math.sqrt(prob["consts"]["mu0"] / prob["consts"]["eps0"])
    amp = max([s["amp"] for s in prob["sources"]] + [0.0])
    if prob.get("e_init") is not None:
        amp = max(amp, float(np.max(np.abs(prob["e_init"]))))
    scale = {"e": amp, "h": amp / eta, "rho": 0.0}
    for r in prob["records"]:
        b = np.asarray(ref[r["name"]])
        if b.size:
            k = _CLASS[r["quantity"]]
            scale[k] = max(scale[k], float(np.max(np.abs(b))))
    return {k: (v if v > 0 else 1.0) for k, v in scale.items()}


def trace_errors(prob, got, ref, n_samples=None):
    """name -> relative error; compares the first n_samples samples when given."""
    scale = class_scales(prob, ref)
    out = {}
    for r in prob["records"]:
        a, b = np.asarray(got[r["name"]]), np.asarray(ref[r["name"]])
        n = len(b) if n_samples is None else min(n_samples, len(a), len(b))
        if n_samples is None and a.shape != b.shape:
            raise ValueError(f"record {r['name']}: shape {a.shape} vs {b.shape}")
        if n == 0:
            out[r["name"]] = 0.0
            continue
        out[r["name"]] = float(np.max(np.abs(a[:n] - b[:n])) / scale[_CLASS[r["quantity"]]])
    return out


def max_error(prob, got, ref, n_samples=None):
    e = trace_errors(prob, got, ref, n_samples)
    return max(e.values()) if e else 0.0
