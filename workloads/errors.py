"""Error measure used to compare recorded traces (no method arithmetic here).

The relative max-norm of each recorded trace: for every record r,

    err_r = max |got_r - ref_r|  /  max( max |ref_r| , FLOOR[quantity of r] ),

i.e. ||x - x_ref||_inf / ||x_ref||_inf per trace (a whole-domain record is one
trace: all its samples of all cells).  The floor only matters for traces whose
reference stays below it, so that a trace that is zero up to rounding is not
divided by its own rounding noise:

* density-matrix quantities (populations, inversions, coherences): 1e-3.  They
  are numbers in [-1, 1] computed with the O(1) elements of the same state, so
  their rounding is absolute, of the size of the state's unit roundoff; a level
  that stays (nearly) empty is measured against 1e-3.
* E: 1 V/m, the smallest field scale of any workload here (the noise that
  starts a laser cavity); H: 1 V/m over the vacuum impedance.

No other scale enters: not the source amplitudes, not the initial field, not
the other traces of the problem.
"""
from __future__ import annotations

import math

import numpy as np

DENSITY_FLOOR = 1e-3
E_FLOOR = 1.0  # V/m


def floor_of(prob, quantity: str) -> float:
    if quantity == "e":
        return E_FLOOR
    if quantity == "h":
        c = prob["consts"]
        return E_FLOOR / math.sqrt(c["mu0"] / c["eps0"])
    return DENSITY_FLOOR


def trace_errors(prob, got, ref, n_samples=None):
    """name -> relative max-norm error of the trace; compares the first n_samples
    samples when given."""
    out = {}
    for r in prob["records"]:
        a, b = np.asarray(got[r["name"]]), np.asarray(ref[r["name"]])
        n = len(b) if n_samples is None else min(n_samples, len(a), len(b))
        if n_samples is None and a.shape != b.shape:
            raise ValueError(f"record {r['name']}: shape {a.shape} vs {b.shape}")
        if n == 0:
            out[r["name"]] = 0.0
            continue
        a, b = a[:n], b[:n]
        scale = max(float(np.max(np.abs(b))), floor_of(prob, r["quantity"]))
        out[r["name"]] = float(np.max(np.abs(a - b)) / scale)
    return out


def max_error(prob, got, ref, n_samples=None):
    e = trace_errors(prob, got, ref, n_samples)
    return max(e.values()) if e else 0.0


def worst(errs):
    """(name, error) of the largest entry of a trace_errors dict."""
    if not errs:
        return ("", 0.0)
    k = max(errs, key=errs.get)
    return (k, errs[k])
