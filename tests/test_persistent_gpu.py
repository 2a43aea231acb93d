"""Persistent (fused multi-step) launch of 1-D lattices and the step-loop autotuner.

The fused kernel runs whole steps with the node state in registers and overlapping
windows of 64 nodes; it must give the separate kernels' results bitwise (same
arithmetic in the same order), for every steps-per-launch and workgroup size, on
the packed C4 columns and on plain D1Q3 grids, and the C4 columns must still match
the oracle after the long run.  The autotuner must leave the state where it was.
"""
import os
import sys

import numpy as np
import pytest

from parity_util import compare
from workloads import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_full_run as mk  # noqa: E402  (case definitions shared with the generator)

KEYS = ("rho_a", "u", "P", "X", "j_a", "rho", "theta")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_02930_amd import lbm as _lbm
    return _lbm, torch


def _log(msg):
    print(msg, flush=True)


def _c4_batch(lbm, stream, cols=None):
    if cols is None:
        cols, _ = mk.c4_columns()
    lengths = [c.nx for c in cols]
    cat = lambda k: np.concatenate([getattr(c, k) for c in cols], axis=-1)
    w0 = cols[0]
    lat = lbm.Lattice(1, int(sum(lengths)), 1, 1, w0.molar_mass, w0.D_ref_lat, cat("X0"), cat("T0"), cat("P0"),
                      T_ref=w0.T_ref, bc_lo=w0.bc_lo, bc_hi=w0.bc_hi, inlet_lo_X=w0.inlet_lo_X,
                      inlet_T=w0.inlet_T, col_len=lengths, stream=stream)
    lat.set_porous_field(cat("phi"), cat("tort"), w0.pore_radius)
    lat.set_faradaic_source(cat("faradaic_rate"), 0, 1)
    lat.set_mechanism(w0.mech)
    return lat


def _fields(lat):
    f = lat.fields()
    return {k: np.asarray(f[k]) for k in KEYS if k in f and np.asarray(f[k]).size}


def _assert_bitwise(a, b, label):
    for k in a:
        if not np.array_equal(a[k], b[k]):
            d = np.max(np.abs(a[k] - b[k]))
            s = np.max(np.abs(a[k]))
            raise AssertionError(f"{label}: field {k} differs, max |diff| {d:.3e} (scale {s:.3e})")


@pytest.mark.parametrize("steps,wpb", [(1, 1), (3, 1), (3, 2), (5, 4), (7, 1)])
def test_fused_c4_columns_bitwise_separate_kernels(env, steps, wpb):
    lbm, torch = env
    stream = torch.cuda.Stream()
    n = 1 + 4 * steps + 2                 # first step, whole launches, a separate-kernel remainder
    _log(f"c4 columns: fused {steps} steps per launch, {wpb} waves per block, {n} steps")
    ref = _c4_batch(lbm, stream.cuda_stream)
    ref.step(n)
    a = _fields(ref)
    ref.close()
    lat = _c4_batch(lbm, stream.cuda_stream)
    lat.set_persistent(steps, wpb)
    lat.step(n)
    b = _fields(lat)
    lat.close()
    _assert_bitwise(a, b, f"fused S={steps} wpb={wpb}")


def test_fused_with_graph_loop_bitwise(env):
    lbm, torch = env
    stream = torch.cuda.Stream()
    n = 1 + 2 * 36 + 3                    # two graph replays of 36 steps (12 launches of 3) and a tail
    ref = _c4_batch(lbm, stream.cuda_stream)
    ref.step(n)
    a = _fields(ref)
    ref.close()
    lat = _c4_batch(lbm, stream.cuda_stream)
    lat.set_persistent(3, 1)
    lat.set_graph(32)
    lat.step(n)
    b = _fields(lat)
    lat.close()
    _assert_bitwise(a, b, "fused S=3 in the graph step loop")


def test_fused_batched_column_equals_column_alone(env):
    lbm, torch = env
    stream = torch.cuda.Stream()
    cols, pick = mk.c4_columns()
    n = 1 + 3 * 5
    lat = _c4_batch(lbm, stream.cuda_stream, cols)
    lat.set_persistent(3, 1)
    lat.step(n)
    f = lat.fields()
    lat.close()
    offs = np.concatenate([[0], np.cumsum([c.nx for c in cols])])
    for c_idx in pick:
        one = lbm.lattice_from_workload(cols[c_idx], stream=stream.cuda_stream)
        one.set_persistent(3, 1)
        one.step(n)
        g = _fields(one)
        one.close()
        sl = slice(int(offs[c_idx]), int(offs[c_idx + 1]))
        _log(f"column {c_idx} (L={cols[c_idx].nx}) alone vs in the batch")
        _assert_bitwise({k: np.asarray(f[k])[..., sl] for k in g}, g, f"column {c_idx}")


@pytest.mark.parametrize("case", ["inlet_outflow_knudsen", "bounceback_both_nochem", "tiny_columns"])
def test_fused_plain_grids_and_edge_cases(env, case):
    lbm, torch = env
    stream = torch.cuda.Stream()
    if case == "tiny_columns":        # columns shorter than the halo, several per window
        cols = [synth.config4_column(L, 0.35 + 0.01 * j, 0.5) for j, L in enumerate([2, 3, 5, 2, 9, 70, 4])]
        mk_lat = lambda: _c4_batch(lbm, stream.cuda_stream, cols)
        n = 1 + 3 * 4
    else:
        w = synth.config4_column(173, 0.4, 1.0)
        if case == "inlet_outflow_knudsen":
            from dataclasses import replace
            w = replace(w, bc_hi=synth.BC_OUTFLOW, mech=None, faradaic_rate=None)
        else:
            from dataclasses import replace
            w = replace(w, bc_lo=synth.BC_BOUNCEBACK, bc_hi=synth.BC_BOUNCEBACK, inlet_lo_X=None, mech=None,
                        faradaic_rate=None, X0=w.X0 * 0 + np.array([0.5, 0.2, 0.1, 0.1, 0.1])[:, None]
                        + 0.05 * np.sin(np.arange(w.nx) / 7.0)[None, :] * np.array([1, -1, 0, 0, 0])[:, None])
        mk_lat = lambda: lbm.lattice_from_workload(w, stream=stream.cuda_stream)
        n = 1 + 5 * 3 + 1
    ref = mk_lat()
    ref.step(n)
    a = _fields(ref)
    ref.close()
    lat = mk_lat()
    lat.set_persistent(5 if case != "tiny_columns" else 3, 1)
    lat.step(n)
    b = _fields(lat)
    lat.close()
    _assert_bitwise(a, b, case)


def test_fused_c4_columns_long_run_against_oracle(env):
    lbm, torch = env
    stream = torch.cuda.Stream()
    path = os.path.join(HERE, "golden", "full_run", "c4_cols.npz")
    g = np.load(path, allow_pickle=False)
    steps = int(g["meta__steps"])
    cols, pick = mk.c4_columns()
    lat = _c4_batch(lbm, stream.cuda_stream, cols)
    lat.set_persistent(3, 1)
    lat.set_graph(32)
    lat.step(steps)
    f = lat.fields()
    lat.close()
    offs = np.concatenate([[0], np.cumsum([c.nx for c in cols])])
    keys = ("rho_a", "u", "P", "X", "j_a", "theta")
    for j, c_idx in enumerate(pick):
        sl = slice(int(offs[c_idx]), int(offs[c_idx + 1]))
        compare({k: np.asarray(f[k])[..., sl] for k in keys}, {k: g[f"col{j}__{k}"] for k in keys}, keys,
                label=f"fused: c4 column {c_idx} after {steps} steps")


def test_autotune_keeps_the_state_and_installs_a_candidate(env):
    lbm, torch = env
    stream = torch.cuda.Stream()
    ref = _c4_batch(lbm, stream.cuda_stream)
    ref.step(1 + 12)
    a = _fields(ref)
    ref.close()
    lat = _c4_batch(lbm, stream.cuda_stream)
    lat.step(1)
    table = lat.autotune(trial_steps=30)
    _log("autotune: " + "; ".join(f"fused={t[0]} chem={t[5]} graph={t[1]} S={t[2]} wpb={t[3]}: {t[4] * 1e3:.1f} us"
                                  for t in table))
    assert len(table) == 9 and all(t[4] > 0 for t in table)
    d = lat.diagnostics(check=False)
    assert d["steps_done"] == 1
    lat.step(12)
    b = _fields(lat)
    lat.close()
    _assert_bitwise(a, b, "after autotune")


def test_chemistry_at_two_waves_per_simd_bitwise(env):
    """The generated chemistry compiled for two waves per SIMD (registers capped, spills to
    scratch) gives the default form's fields bitwise, on the C4 columns and a C3 sub-grid."""
    lbm, torch = env
    stream = torch.cuda.Stream()
    ref = _c4_batch(lbm, stream.cuda_stream)
    ref.step(12)
    a = _fields(ref)
    ref.close()
    lat = _c4_batch(lbm, stream.cuda_stream)
    lat.set_chem_kernel(lbm.CHEM_SPECIALIZED_2W)
    lat.step(12)
    b = _fields(lat)
    lat.close()
    _assert_bitwise(a, b, "c4 columns, chemistry at two waves per SIMD")
    w = synth.config3(nx=32, ny=16, nz=16)
    runs = []
    for kind in (lbm.CHEM_SPECIALIZED, lbm.CHEM_SPECIALIZED_2W):
        lat = lbm.lattice_from_workload(w, stream=stream.cuda_stream)
        lat.set_chem_kernel(kind)
        lat.step(6)
        runs.append(_fields(lat))
        lat.close()
    _assert_bitwise(runs[0], runs[1], "c3 32x16x16, chemistry at two waves per SIMD")
