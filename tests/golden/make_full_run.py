"""Writes the expected fields of the long parity runs (tests/golden/full_run/*.npz).

Calls only the CPU oracle (oracle/) on the seeded inputs of workloads/synth.py; the
GPU tests in tests/test_full_run_gpu.py run the same workloads through the C ABI and
compare.  Each case stores, per output field, the oracle's values at a fixed set of
nodes (all nodes of the 1-D cases) and the field's maximum magnitude over the whole
domain (the scale of the normwise error).

    python tests/golden/make_full_run.py [case ...]       # default: every case
    python tests/golden/make_full_run.py --list

Cases (sizes chosen so the oracle finishes in minutes on the host's cores):
  c2_kn0..c2_kn7   C2 capillary physics (pure H2 | pure N2 inlets, energy on, phi 0.5),
                   one of the 8 Knudsen numbers, 20000 steps, on 128 x 1 (the 128 x 64 GPU run
                   is y-uniform): the capillary at 128 nodes, where the run stays bounded;
                   at the stated 1024 nodes the nearly pure species next to each inlet
                   (beta_a -> 0, an almost collisionless species lattice) diverge
  c5_1024x16       C5 physics (GRF porosity, inlet / outflow, Knudsen) on 1024 x 16,
                   2000 steps, and the objective J of the outlet flux over those steps
  c3_64x32x32      C3 physics (GRF porosity, 10 surface species, 20 reactions) on a
                   64 x 32 x 32 sub-grid, 20 steps
  c3_16x16x16      the same on 16 x 16 x 16, 300 steps
  c3_128x16x8      the same on 128 x 16 x 8, 100 steps (rows of two 64-node tiles, y a
                   multiple of 8: the species kernel's two-tile blocks and XCD y slabs)
  c3_full_sampled  C3 at 256 x 128 x 128, 10 steps, 4 sampled nodes (periodic patches
                   of radius 21 cut around them reproduce the full run there exactly)
  c4_cols          three of the 64 C4 columns (first, longest, last), 500 steps
  c3_energy_16     C3 physics with the energy lattice and adsorbed-phase thermo (synth.config3_energy)
                   on 16 x 16 x 16, 100 steps
"""
import math
import os
import sys
import time
from dataclasses import replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.lbm_oracle import Oracle  # noqa: E402
from workloads import synth  # noqa: E402

OUT = os.path.join(HERE, "full_run")
KEYS = ("rho_a", "u", "T", "P", "X", "j_a", "rho", "theta")
N_SAMPLE = 1024


def sample_nodes(N, n=N_SAMPLE, seed=0):
    """Nodes whose values are stored: all of them for small domains, else a seeded set
    that always includes the first and last node."""
    if N <= n:
        return np.arange(N)
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, N - 1], rng.choice(N, n - 2, replace=False)]))
    return idx


def _store(name, fields, nodes, meta):
    os.makedirs(OUT, exist_ok=True)
    arrs = {"nodes": nodes}
    for k in KEYS:
        if k not in fields:
            continue
        a = np.asarray(fields[k], dtype=np.float64)
        if a.size == 0:
            continue
        arrs[f"{k}__scale"] = np.array(float(np.max(np.abs(a))))
        arrs[k] = a[..., nodes]
    for k, v in meta.items():
        arrs[f"meta__{k}"] = np.array(v)
    np.savez_compressed(os.path.join(OUT, f"{name}.npz"), **arrs)


C2_NX = 128


def case_c2(kn):
    w = synth.config2(kn_index=kn, nx=C2_NX, ny=1)
    o = Oracle(w)
    o.step(20000)
    _store(f"c2_kn{kn}", o.moments(), np.arange(w.N), {"steps": 20000, "kn_index": kn})


def case_c5():
    w = synth.config5(nx=1024, ny=16)
    o = Oracle(w)
    J = o.outlet_flux(2000, species=0)
    _store("c5_1024x16", o.moments(), sample_nodes(w.N), {"steps": 2000, "J": J})


def case_c3(nx, ny, nz, steps):
    w = synth.config3(nx=nx, ny=ny, nz=nz)
    o = Oracle(w)
    o.step(steps)
    _store(f"c3_{nx}x{ny}x{nz}", o.moments(), sample_nodes(w.N), {"steps": steps})


def patch(w, center, R):
    """Periodic patch of radius R around center (x, y, z) cut from workload w, and the
    patch index of its centre.  After k steps a node depends on the initial state within
    radius 2k (pull and gradient stencil), so R >= 2k + 1 reproduces the full run there."""
    n = 2 * R + 1
    off = np.arange(-R, R + 1)
    xs = (center[0] + off) % w.nx
    ys = (center[1] + off) % w.ny if w.lattice > 1 else np.zeros(1, int)
    zs = (center[2] + off) % w.nz if w.lattice > 2 else np.zeros(1, int)
    idx = (xs[None, None, :] + w.nx * (ys[None, :, None] + w.ny * zs[:, None, None])).reshape(-1)
    pw = replace(w, nx=n, ny=n if w.lattice > 1 else 1, nz=n if w.lattice > 2 else 1,
                 X0=w.X0[:, idx], P0=w.P0[idx], T0=w.T0[idx], phi=w.phi[idx], tort=w.tort[idx],
                 bc_lo=synth.BC_PERIODIC, bc_hi=synth.BC_PERIODIC, inlet_lo_X=None, inlet_hi_X=None)
    c = R + n * (R + (n * R if w.lattice > 2 else 0)) if w.lattice > 1 else R
    return pw, c


C3_FULL_CENTERS = [(0, 0, 0), (255, 127, 127), (128, 64, 64), (37, 101, 5)]
C3_FULL_STEPS = 10


def case_c3_full_node(i):
    w = synth.config3()
    ctr = C3_FULL_CENTERS[i]
    pw, c = patch(w, ctr, 2 * C3_FULL_STEPS + 1)
    o = Oracle(pw)
    o.step(C3_FULL_STEPS)
    m = o.moments()
    return {k: np.asarray(v)[..., c] for k, v in m.items() if k in KEYS}


def case_c3_full():
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=len(C3_FULL_CENTERS)) as ex:
        res = list(ex.map(case_c3_full_node, range(len(C3_FULL_CENTERS))))
    w = synth.config3()
    nodes = np.array([c[0] + w.nx * (c[1] + w.ny * c[2]) for c in C3_FULL_CENTERS])
    arrs = {"nodes": nodes}
    for k in res[0]:
        arrs[k] = np.stack([r[k] for r in res], axis=-1)
    for k, v in {"steps": C3_FULL_STEPS}.items():
        arrs[f"meta__{k}"] = np.array(v)
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(os.path.join(OUT, "c3_full_sampled.npz"), **arrs)


C4_STEPS = 500


def c4_columns():
    lengths, phis, currents = synth.config4_columns()
    cols = [synth.config4_column(int(L), float(p), float(i)) for L, p, i in zip(lengths, phis, currents)]
    pick = (0, int(np.argmax(lengths)), len(cols) - 1)
    return cols, pick


def case_c4_col(c_idx):
    cols, _ = c4_columns()
    o = Oracle(cols[c_idx])
    o.step(C4_STEPS)
    return {k: np.asarray(v) for k, v in o.moments().items() if k in KEYS}


def case_c4():
    from concurrent.futures import ProcessPoolExecutor
    _, pick = c4_columns()
    with ProcessPoolExecutor(max_workers=3) as ex:
        res = list(ex.map(case_c4_col, pick))
    arrs = {"meta__steps": np.array(C4_STEPS), "meta__columns": np.array(pick)}
    for j, (c_idx, r) in enumerate(zip(pick, res)):
        for k, v in r.items():
            if v.size:
                arrs[f"col{j}__{k}"] = v
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(os.path.join(OUT, "c4_cols.npz"), **arrs)


def case_c3_energy():
    w = synth.config3_energy(nx=16, ny=16, nz=16)
    o = Oracle(w)
    o.step(100)
    _store("c3_energy_16", o.moments(), sample_nodes(w.N), {"steps": 100})


CASES = {f"c2_kn{k}": (lambda k=k: case_c2(k)) for k in range(8)}
CASES.update({
    "c5_1024x16": case_c5,
    "c3_64x32x32": lambda: case_c3(64, 32, 32, 20),
    "c3_16x16x16": lambda: case_c3(16, 16, 16, 300),
    "c3_128x16x8": lambda: case_c3(128, 16, 8, 100),
    "c3_full_sampled": case_c3_full,
    "c4_cols": case_c4,
    "c3_energy_16": case_c3_energy,
})


def main(argv):
    if "--list" in argv:
        print("\n".join(CASES))
        return
    names = [a for a in argv if not a.startswith("-")] or list(CASES)
    for name in names:
        t0 = time.time()
        CASES[name]()
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
