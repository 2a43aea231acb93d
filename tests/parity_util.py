"""Normwise comparison of GPU fields with the oracle's (shared by the GPU tests).

Every field is compared as max_x |gpu - oracle| / max_x |oracle| (the relative error
of the whole field, reading R23) and must stay within TOL = 1e-11.

Velocity-like fields are differences of populations: u = sum_i f_i c_i / rho and the
species momenta j_a come from sums whose terms are of the size of the populations
(sum_i |f_i c_i| <= phi rho, resp. phi rho_a), so computed in two summation orders
they differ by some ulps of that scale however small the field itself is (a closed
cell where only the reactions move the gas has max |u| ~ 1e-8 at rest-like states:
there 1e-11 of the field is 1e-19, below one ulp of the populations).  Such a field
passes when it is within TOL relative, or else within ROUND_ULPS ulps of its
population scale (u: 1; j_a: max rho_a); the comparison prints which fields needed
that bound and by how much they missed the relative one.  No other field has a
floor.
"""
import sys

import numpy as np

TOL = 1e-11
EPS = float(np.finfo(np.float64).eps)
ROUND_ULPS = 64.0
POP_SCALED = ("u", "j_a")


def population_scale(key, ref):
    if key == "u":
        return 1.0
    if key == "j_a":
        ra = ref.get("rho_a") if isinstance(ref, dict) else None
        return float(np.max(np.abs(ra))) if ra is not None else 30.0
    return None


def field_error(g, r):
    """(relative error, absolute error) of a field."""
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    r = np.asarray(r, dtype=np.float64).reshape(-1)
    assert g.shape == r.shape, (g.shape, r.shape)
    assert np.all(np.isfinite(g))
    if r.size == 0:
        return 0.0, 0.0
    diff = float(np.max(np.abs(g - r)))
    scale = float(np.max(np.abs(r)))
    rel = diff / scale if scale > 0 else (0.0 if diff == 0 else np.inf)
    return rel, diff


def check_field(key, g, r, ref=None, tol=TOL):
    """Returns (passed, rel, abs, used_roundoff_bound)."""
    rel, diff = field_error(g, r)
    if rel <= tol:
        return True, rel, diff, False
    s = population_scale(key, ref or {}) if key in POP_SCALED else None
    if s is not None and diff <= ROUND_ULPS * EPS * s:
        return True, rel, diff, True
    return False, rel, diff, False


def compare(got, ref, keys, tol=TOL, label=""):
    """Asserts every field; returns the relative errors and prints them."""
    errs, rb, bad = {}, {}, {}
    for k in keys:
        ok, rel, diff, used = check_field(k, np.asarray(got[k]), np.asarray(ref[k]), ref, tol)
        errs[k] = rel
        if used:
            rb[k] = diff
        if not ok:
            bad[k] = (rel, diff)
    msg = f"{label} relative errors {errs}"
    if rb:
        msg += f"; within {ROUND_ULPS:g} ulps of the population scale instead: {rb}"
    print(msg, flush=True)
    sys.stdout.flush()
    assert not bad, f"{label}: fields off (relative, absolute): {bad} (all: {errs})"
    return errs


def normalized_error(g, r, key=None, ref=None, tol=TOL):
    """An error that is <= tol exactly when check_field passes (for `assert err <= tol`)."""
    ok, rel, diff, used = check_field(key, g, r, ref, tol)
    if used:
        return tol
    return rel
