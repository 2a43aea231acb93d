"""Parity after the long runs: the GPU path through the C ABI against the oracle's
fields stored by tests/golden/make_full_run.py (which calls only the oracle).

C2 physics (pure-species inlets, energy on) for the stated 20000 steps at each of the 8
Knudsen numbers, on 128 x 64 nodes (at the stated 1024 x 64 the scheme diverges, on
the oracle and the GPU alike); the run is y-uniform, so its rows are compared with the
oracle's 128 x 1 run.  C5 physics (GRF porosity, Knudsen drag,
inlet / outflow) on 1024 x 16 for 2000 steps, with the outlet-flux objective over
the run.  C3 physics on 64 x 32 x 32 (20 steps), 16 x 16 x 16 (300 steps) and 128 x 16 x 8
(100 steps: the two-tile species blocks with the XCD y-slab walk of the full grid), and C3
at its full size 256 x 128 x 128 after 10 steps at 4 sampled nodes.  Three of the 64
batched C4 columns after 500 steps.  C3 physics with the energy lattice on 16 x 16 x 16 for 100
steps.  Every field within 1e-11 normwise (parity_util).
"""
import os
import sys

import numpy as np
import pytest

from parity_util import compare
from workloads import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "full_run")
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_full_run as mk  # noqa: E402  (case definitions shared with the generator)


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_02930_amd import lbm as _lbm
    return _lbm


def _gold(name):
    path = os.path.join(GOLD, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated (python tests/golden/make_full_run.py {name})")
    return np.load(path, allow_pickle=False)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kn", range(8))
def test_c2_capillary_full_run_every_knudsen_number(lbm, kn):
    g = _gold(f"c2_kn{kn}")
    steps = int(g["meta__steps"])
    w = synth.config2(kn_index=kn, nx=mk.C2_NX)
    _log(f"c2 kn index {kn}: {w.nx}x{w.ny}, {steps} steps")
    lat = lbm.lattice_from_workload(w)
    lat.step(steps)
    f = lat.fields()
    lat.close()
    keys = ("rho_a", "u", "T", "P", "X", "j_a", "rho")
    got = {k: np.asarray(f[k]).reshape(np.asarray(f[k]).shape[:-1] + (w.ny, w.nx)) for k in keys}
    for row in (0, w.ny // 2, w.ny - 1):
        compare({k: got[k][..., row, :] for k in keys}, {k: g[k] for k in keys}, keys,
                label=f"c2 kn{kn} row {row}")
    # y-uniformity of the GPU run: every row equals row 0
    for k in keys:
        a = got[k]
        assert np.max(np.abs(a - a[..., :1, :])) <= 1e-13 * max(np.max(np.abs(a)), 1e-300), k


def test_c5_full_run_on_reduced_width_with_outlet_flux(lbm):
    g = _gold("c5_1024x16")
    steps = int(g["meta__steps"])
    w = synth.config5(nx=1024, ny=16)
    lat = lbm.lattice_from_workload(w)
    lat.step(steps)
    f = lat.fields()
    lat.close()
    nodes = g["nodes"]
    keys = ("rho_a", "u", "P", "X", "j_a", "rho")
    compare({k: np.asarray(f[k])[..., nodes] for k in keys}, {k: g[k] for k in keys}, keys,
            label=f"c5 1024x16 after {steps} steps")
    lat = lbm.lattice_from_workload(w)
    J, _, _ = lat.adjoint_outlet_flux(steps, 0)
    lat.close()
    Jref = float(g["meta__J"])
    _log(f"c5 outlet flux J gpu {J!r} oracle {Jref!r}")
    assert abs(J - Jref) <= 1e-11 * abs(Jref)


@pytest.mark.parametrize("shape", ["64x32x32", "16x16x16", "128x16x8"])
def test_c3_sub_grid_full_run(lbm, shape):
    g = _gold(f"c3_{shape}")
    steps = int(g["meta__steps"])
    nx, ny, nz = (int(v) for v in shape.split("x"))
    w = synth.config3(nx=nx, ny=ny, nz=nz)
    lat = lbm.lattice_from_workload(w)
    lat.step(steps)
    f = lat.fields()
    d = lat.diagnostics(check=False)
    lat.close()
    assert d["n_nonfinite"] == 0
    nodes = g["nodes"]
    keys = ("rho_a", "u", "P", "X", "j_a", "rho", "theta")
    compare({k: np.asarray(f[k])[..., nodes] for k in keys}, {k: g[k] for k in keys}, keys,
            label=f"c3 {shape} after {steps} steps")


def test_c3_full_size_ten_steps_sampled(lbm):
    g = _gold("c3_full_sampled")
    steps = int(g["meta__steps"])
    w = synth.config3()
    lat = lbm.lattice_from_workload(w)
    lat.step(steps)
    f = lat.fields()
    lat.close()
    nodes = g["nodes"]
    keys = ("rho_a", "u", "P", "X", "j_a", "rho", "theta")
    compare({k: np.asarray(f[k])[..., nodes] for k in keys}, {k: g[k] for k in keys}, keys,
            label=f"c3 256x128x128 after {steps} steps, {nodes.size} sampled nodes")


def test_c4_batched_columns_long_run(lbm):
    import torch
    stream = torch.cuda.Stream()                     # the graph step loop runs on a stream of its own
    g = _gold("c4_cols")
    steps = int(g["meta__steps"])
    cols, pick = mk.c4_columns()
    lengths = [c.nx for c in cols]
    cat = lambda k: np.concatenate([getattr(c, k) for c in cols], axis=-1)
    w0 = cols[0]
    lat = lbm.Lattice(1, int(sum(lengths)), 1, 1, w0.molar_mass, w0.D_ref_lat, cat("X0"), cat("T0"), cat("P0"),
                      T_ref=w0.T_ref, bc_lo=w0.bc_lo, bc_hi=w0.bc_hi, inlet_lo_X=w0.inlet_lo_X,
                      inlet_T=w0.inlet_T, col_len=lengths, stream=stream.cuda_stream)
    lat.set_porous_field(cat("phi"), cat("tort"), w0.pore_radius)
    lat.set_faradaic_source(cat("faradaic_rate"), 0, 1)
    lat.set_mechanism(w0.mech)
    lat.set_graph(32)
    lat.step(steps)
    f = lat.fields()
    lat.close()
    offs = np.concatenate([[0], np.cumsum(lengths)])
    keys = ("rho_a", "u", "P", "X", "j_a", "theta")
    for j, c_idx in enumerate(pick):
        sl = slice(int(offs[c_idx]), int(offs[c_idx + 1]))
        compare({k: np.asarray(f[k])[..., sl] for k in keys}, {k: g[f"col{j}__{k}"] for k in keys}, keys,
                label=f"c4 column {c_idx} (L={lengths[c_idx]}) after {steps} steps")


def test_c3_energy_full_run(lbm):
    """C3 physics with the energy lattice and adsorbed-phase thermo (the surface chemistry moving
    internal energy between the phases) on 16 x 16 x 16 for 100 steps."""
    g = _gold("c3_energy_16")
    steps = int(g["meta__steps"])
    w = synth.config3_energy(nx=16, ny=16, nz=16)
    lat = lbm.lattice_from_workload(w)
    lat.step(steps)
    f = lat.fields()
    d = lat.diagnostics(check=False)
    lat.close()
    assert d["n_nonfinite"] == 0
    nodes = g["nodes"]
    keys = ("rho_a", "u", "T", "P", "X", "j_a", "rho", "theta")
    compare({k: np.asarray(f[k])[..., nodes] for k in keys}, {k: g[k] for k in keys}, keys,
            label=f"c3 energy 16x16x16 after {steps} steps")
