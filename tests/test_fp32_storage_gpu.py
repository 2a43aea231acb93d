"""FP32 population storage (lbm_config.precision = LBM_FP32): every population is
rounded to FP32 (unit roundoff u = 2^-24) when it is stored, all arithmetic is
FP64.  Each step stores each population once, so after n steps the populations
carry at most about n rounding errors of relative size u each; moments are
sums of at most (M+2)Q populations of one sign pattern, so their relative
error is bounded by the same order.  The test bound is n * u * 16 (a factor 16
over the one-rounding-per-step estimate for the growth of the errors through
the collision), checked against the FP64 oracle field by field, normwise as in
the FP64 parity tests.  The measured errors are printed."""
import sys

import numpy as np

from parity_util import POP_SCALED, population_scale
import pytest

from oracle.lbm_oracle import Oracle
from workloads import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_02930_amd import lbm as _lbm
    return _lbm


def _errs(got, ref, keys):
    """Normwise relative error per field; for u and j_a, differences of populations,
    the absolute error in units of their population scale (1, resp. max rho_a) when
    that is the smaller: FP32 rounding of the stored populations is relative to the
    populations, not to the (much smaller) velocities they cancel down to."""
    out = {}
    for k in keys:
        g = np.asarray(got[k], dtype=np.float64).reshape(-1)
        r = np.asarray(ref[k], dtype=np.float64).reshape(-1)
        assert g.shape == r.shape and np.all(np.isfinite(g)), k
        scale = float(np.max(np.abs(r)))
        diff = float(np.max(np.abs(g - r)))
        e = 0.0 if scale == 0 else diff / scale
        s = population_scale(k, ref) if k in POP_SCALED else None
        out[k] = min(e, diff / s) if s else e
    return out


CASES = {
    "c1_d2q9": (lambda: synth.config1(nx=12, ny=8), 100),
    "c2_energy_inlets": (lambda: synth.config2(kn_index=3, nx=64, ny=4), 150),
    "c3_d3q27_chemistry": (lambda: synth.config3(nx=10, ny=6, nz=4), 12),
    "c3_row_blocks": (lambda: synth.config3(nx=64, ny=3, nz=8), 6),
    "c3_two_tile_xcd_slabs": (lambda: synth.config3(nx=128, ny=8, nz=3), 6),
    "electrode_current_control": (lambda: _controlled(synth.electrode_slab(nx=16, ny=2, omega=5e-3)), 20),
}


def _controlled(w):
    w.electrode["target_ia"] = np.array([1.0e6, 1.5e6])
    w.electrode["n_secant"] = 6
    return w


@pytest.mark.parametrize("case", list(CASES))
def test_fp32_storage_against_oracle(lbm, case):
    make, steps = CASES[case]
    w = make()
    keys = ["rho_a", "u", "T", "P", "j_a", "X", "rho"] + (["theta"] if w.mech is not None else [])
    print(f"case {case} N={w.N} steps={steps}", flush=True)
    lat = lbm.lattice_from_workload(w, precision=lbm.FP32)
    lat.step(steps)
    got = lat.fields()
    d = lat.diagnostics(check=False)
    lat.close()
    assert d["n_nonfinite"] == 0
    o = Oracle(w)
    o.step(steps)
    ref = o.moments()
    errs = _errs(got, ref, keys)
    tol = steps * U32 * 16
    print(f"{case}: FP32 storage vs FP64 oracle after {steps} steps, bound {tol:.2e}: {errs}", flush=True)
    sys.stdout.flush()
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, bad
    # the storage really is FP32: the run differs from the FP64 one by more than FP64 rounding
    lat64 = lbm.lattice_from_workload(w)
    lat64.step(steps)
    f64 = lat64.fields()
    lat64.close()
    assert max(_errs(got, f64, ["rho_a", "P"]).values()) > 1e-12


def test_fp32_snapshot_roundtrip_bitwise(lbm):
    w = synth.config3(nx=9, ny=5, nz=3)
    a = lbm.lattice_from_workload(w, precision=lbm.FP32)
    a.step(4)
    blob = a.save()
    a.step(4)
    fa = a.fields()
    b = lbm.lattice_from_workload(w, precision=lbm.FP32)
    b.load(blob)
    b.step(4)
    fb = b.fields()
    for k in fa:
        assert np.array_equal(np.asarray(fa[k]), np.asarray(fb[k])), k
    a.close()
    b.close()
    c = lbm.lattice_from_workload(w)          # FP64 context refuses an FP32 snapshot
    with pytest.raises(lbm.LBMError):
        c.load(blob)
    c.close()
