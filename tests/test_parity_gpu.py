"""HIP path vs the FP64 oracle on the same seeded inputs (through the C ABI).

Fields are compared per output field with the normwise relative error
max_x |gpu - oracle| / max_x |oracle| <= 1e-11 (FP64 on both sides; the two differ
only by rounding order, FMA contraction and libm ulps, and every run here is
dissipative), with no per-field floor; only the velocity-like fields u and j_a,
differences of populations, may instead sit within 64 ulps of their population
scale when they are themselves far below it (parity_util says which and why).
"""
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle.lbm_oracle import Oracle
from workloads import synth

pytestmark = pytest.mark.gpu

from parity_util import TOL, compare as _pcompare


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_02930_amd import lbm as _lbm
    return _lbm


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(got, ref, keys, tol=TOL, label=""):
    return _pcompare(got, ref, keys, tol=tol, label=label)


def _run(lbm, w, steps, keys=("rho_a", "u", "T", "P", "j_a", "X", "rho"), chem_kernel=None):
    _log(f"case {w.name} N={w.N} steps={steps} chem_kernel={chem_kernel}")
    lat = lbm.lattice_from_workload(w)
    if chem_kernel is not None:
        lat.set_chem_kernel(chem_kernel)
    lat.step(steps)
    got = lat.fields()
    lat.close()
    o = Oracle(w)
    o.step(steps)
    ref = o.moments()
    keys = list(keys) + (["theta"] if w.mech is not None else [])
    return _compare(got, ref, keys)


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_first_steps_tiny(lbm, steps):
    w = synth.config1(nx=12, ny=8)
    _run(lbm, w, steps)


def test_c1_full_run(lbm):
    """Config 1 as stated: D2Q9 64x64 periodic, 1000 steps."""
    w = synth.config1()
    _run(lbm, w, w.steps)


def test_c1_ragged_grid_knudsen_off(lbm):
    w = synth.config1(nx=37, ny=23, pore_radius=float("inf"))
    _run(lbm, w, 150)


def test_d1q3_three_species(lbm):
    w = synth.config5(nx=301, ny=4)
    w = replace(w, lattice=1, ny=1, X0=w.X0[:, :301], P0=w.P0[:301], T0=w.T0[:301], phi=w.phi[:301],
                tort=w.tort[:301], bc_lo=synth.BC_PERIODIC, bc_hi=synth.BC_PERIODIC)
    _run(lbm, w, 120)


def test_d3q27_porous_no_chemistry(lbm):
    w = synth.config3(nx=13, ny=7, nz=5, with_mech=False)
    _run(lbm, w, 40)


@pytest.mark.parametrize("kernel", ["specialized", "generic"])
def test_d3q27_porous_with_chemistry(lbm, kernel):
    w = synth.config3(nx=10, ny=6, nz=4)
    kind = lbm.CHEM_SPECIALIZED if kernel == "specialized" else lbm.CHEM_GENERIC
    _run(lbm, w, 12, chem_kernel=kind)


@pytest.mark.parametrize("shape", [(64, 3, 8), (128, 2, 16), (128, 8, 6), (256, 16, 3)])
def test_d3q27_row_blocks_with_chemistry(lbm, shape):
    """Rows that are whole 64-node tiles: the species kernel stages the
    previous step's records of the 3 x 3 neighbouring rows in LDS (periodic
    wrap at the row ends, two tiles per row in the second case).  In the last two
    shapes (ny a multiple of 8, rows of whole two-tile blocks) each XCD walks
    its own y slab of every z plane."""
    nx, ny, nz = shape
    w = synth.config3(nx=nx, ny=ny, nz=nz)
    _run(lbm, w, 6)


@pytest.mark.parametrize("kernel", ["specialized", "generic"])
def test_d3q27_energy_with_chemistry(lbm, kernel):
    """Energy lattice with the surface mechanism and adsorbed-phase thermo: the
    chemistry's energy source (unified internal energy kept, g^eq,source)."""
    w = synth.config3_energy(nx=10, ny=6, nz=4)
    kind = lbm.CHEM_SPECIALIZED if kernel == "specialized" else lbm.CHEM_GENERIC
    _run(lbm, w, 8, chem_kernel=kind)


def test_d3q27_inlet_outflow_chemistry_xcd_slabs(lbm):
    """C3 physics with an inlet of another composition at x = 0 and an outflow at
    x = nx - 1 on a grid where the species kernel runs two tiles per block and the
    XCD y-slab walk: the x-end tiles gather their reaction populations directly,
    the interior row tiles stage them."""
    w = synth.config3(nx=256, ny=8, nz=2)
    w = replace(w, bc_lo=synth.BC_INLET, bc_hi=synth.BC_OUTFLOW,
                inlet_lo_X=np.array([0.6, 0.1, 0.1, 0.1, 0.1]), inlet_T=float(w.T0[0]))
    _run(lbm, w, 6)


def test_d3q27_energy_xcd_slabs(lbm):
    """Energy lattice (one tile per block) on a grid whose y extent is a multiple of
    8 and whose rows hold whole tiles: the XCD y-slab walk of the species kernel."""
    w = synth.config3_energy(nx=64, ny=8, nz=3)
    _run(lbm, w, 6)


def _uniform_phi(w, phi):
    return replace(w, phi=np.full(w.N, phi), tort=np.full(w.N, phi ** -0.5))


DEGENERATE = {
    "d2q9_single_node": lambda: synth.config1(nx=1, ny=1),
    "d3q27_single_node_chemistry": lambda: _uniform_phi(synth.config3(nx=1, ny=1, nz=1), 0.45),
    "d3q27_3x1x2_chemistry": lambda: _uniform_phi(synth.config3(nx=3, ny=1, nz=2), 0.4),
    "d1q3_two_node_column": lambda: synth.config4_column(2, 0.4, 1.0),
}


@pytest.mark.parametrize("case", list(DEGENERATE))
def test_degenerate_grids(lbm, case):
    """One node (every direction streams back onto it), a grid thinner than the
    stencil in y, a two-node column with an inlet and a wall at its ends."""
    _run(lbm, DEGENERATE[case](), 5)


HOMOGENEOUS = {
    "d1q3_dimerisation": lambda: synth.homogeneous_dimerisation(nx=8),
    "d2q9_dimerisation_and_adsorption": lambda: synth.homogeneous_dimerisation(nx=6, ny=4, with_surface=True),
}


@pytest.mark.parametrize("kernel", ["specialized", "generic"])
@pytest.mark.parametrize("case", list(HOMOGENEOUS))
def test_homogeneous_gas_reactions(lbm, case, kernel):
    """Homogeneous gas-phase reaction 2A <=> B alone and next to a surface
    reaction (eqs sumRhoDot, totalFluidReactionRate)."""
    kind = lbm.CHEM_SPECIALIZED if kernel == "specialized" else lbm.CHEM_GENERIC
    _run(lbm, HOMOGENEOUS[case](), 20, chem_kernel=kind)


TWO_PHASE = {
    "edge_transfer_only": lambda: synth.two_phase_tpb(nx=5, ny=3, with_gas=False),
    "adsorption_edge_desorption": lambda: synth.two_phase_tpb(nx=6, ny=4, with_gas=True),
}


@pytest.mark.parametrize("kernel", ["specialized", "generic"])
@pytest.mark.parametrize("case", list(TWO_PHASE))
def test_two_surface_phases_with_tpb_edge(lbm, case, kernel):
    """Electrode and electrolyte surfaces with their own site densities and areas,
    joined by a TPB edge reaction (eqs totalSurfaceReactionRateTPB_electrode and
    _electrolyte)."""
    kind = lbm.CHEM_SPECIALIZED if kernel == "specialized" else lbm.CHEM_GENERIC
    _run(lbm, TWO_PHASE[case](), 20, chem_kernel=kind)


def test_specialized_chemistry_matches_generic_full_newton(lbm):
    """Specialised vs generic kernel on a stiffer mechanism setting (more
    sub-steps and Newton iterations), both through lbm_step: every field
    agrees to rounding."""
    w = synth.config3(nx=12, ny=8, nz=6)
    w = replace(w, mech=replace(w.mech, n_sub=3, n_newton=4))
    out = {}
    for kind in (lbm.CHEM_GENERIC, lbm.CHEM_SPECIALIZED):
        lat = lbm.lattice_from_workload(w)
        lat.set_chem_kernel(kind)
        lat.step(8)
        out[kind] = lat.fields()
        lat.close()
    _compare(out[lbm.CHEM_SPECIALIZED], out[lbm.CHEM_GENERIC], ("rho_a", "u", "P", "j_a", "theta"), tol=1e-12)


def test_c2_energy_inlets_short(lbm):
    w = synth.config2(kn_index=3, nx=64, ny=4)
    _run(lbm, w, 150)


def test_c5_inlet_outflow_grf(lbm):
    w = synth.config5(nx=48, ny=16)
    _run(lbm, w, 120)


def test_c4_columns_match_oracle_and_plain(lbm):
    lengths = [30, 45, 17]
    phis = [0.35, 0.45, 0.3]
    cur = [0.0, 1.0, 2.0]
    cols = [synth.config4_column(L, p, i, n_sub=2, n_newton=3) for L, p, i in zip(lengths, phis, cur)]
    steps = 40
    # batched packed run
    cat = lambda k: np.concatenate([getattr(c, k) for c in cols], axis=-1)
    w0 = cols[0]
    lat = lbm.Lattice(1, int(sum(lengths)), 1, 1, w0.molar_mass, w0.D_ref_lat, cat("X0"), cat("T0"), cat("P0"),
                      T_ref=w0.T_ref, bc_lo=w0.bc_lo, bc_hi=w0.bc_hi, inlet_lo_X=w0.inlet_lo_X,
                      inlet_T=w0.inlet_T, col_len=lengths)
    lat.set_porous_field(cat("phi"), cat("tort"), w0.pore_radius)
    lat.set_faradaic_source(cat("faradaic_rate"), 0, 1)
    lat.set_mechanism(w0.mech)
    lat.set_chem_kernel(lbm.CHEM_GENERIC)     # node-local and order-independent: batched == plain bitwise
    lat.step(steps)
    got = lat.fields()
    lat.close()
    off = 0
    for c in cols:
        _log(f"column L={c.nx}")
        plain = lbm.lattice_from_workload(c)
        plain.set_chem_kernel(lbm.CHEM_GENERIC)
        plain.step(steps)
        gp = plain.fields()
        plain.close()
        sl = slice(off, off + c.nx)
        for k in ("rho_a", "u", "P", "theta", "X"):
            a = np.asarray(got[k])[..., sl]
            b = np.asarray(gp[k])
            assert np.array_equal(a, b), k          # batched == plain, bitwise
        o = Oracle(c)
        o.step(steps)
        ref = o.moments()
        _compare(gp, ref, ("rho_a", "u", "P", "X", "j_a", "theta"))
        spec = lbm.lattice_from_workload(c)       # default: specialised chemistry
        spec.step(steps)
        _compare(spec.fields(), ref, ("rho_a", "u", "P", "X", "j_a", "theta"))
        spec.close()
        off += c.nx


def test_conservation_on_gpu(lbm):
    w = synth.config1(nx=96, ny=80, pore_radius=float("inf"))
    lat = lbm.lattice_from_workload(w)
    d0 = lat.diagnostics()
    lat.step(500)
    d1 = lat.diagnostics()
    rel = np.abs(d1["species_mass"] - d0["species_mass"]) / d0["species_mass"]
    assert np.all(rel < 1e-13), rel
    assert abs(d1["mixture_mass"] - d0["mixture_mass"]) / d0["mixture_mass"] < 1e-13
    assert np.all(np.abs(d1["mixture_momentum"]) < 1e-13 * d0["mixture_mass"])
    lat.close()


def test_diagnostics_include_pending_reaction_populations(lbm):
    """The last step's reaction populations live in the node records until the
    next pull; the diagnostics must count them.  With periodic boundaries the
    stream is a permutation, so the oracle's post-stream totals and minimum
    equal the stored (pre-stream) ones."""
    w = synth.config3(nx=9, ny=5, nz=3)
    assert w.bc_lo == synth.BC_PERIODIC and w.bc_hi == synth.BC_PERIODIC
    lat = lbm.lattice_from_workload(w)
    lat.step(4)
    d = lat.diagnostics()
    lat.close()
    o = Oracle(w)
    o.step(4)
    mass = o.fa.sum(axis=(1, 2))
    rel = np.abs(d["species_mass"] - mass) / mass
    assert np.all(rel < 1e-12), rel
    ref_min = min(float(o.fa.min()), float(o.f.min()))
    assert abs(d["min_population"] - ref_min) <= 1e-11 * abs(ref_min), (d["min_population"], ref_min)


def test_save_load_roundtrip_bitwise(lbm):
    w = synth.config3(nx=9, ny=5, nz=3)
    a = lbm.lattice_from_workload(w)
    a.step(6)
    blob = a.save()
    a.step(6)
    fa = a.fields()
    b = lbm.lattice_from_workload(w)
    b.load(blob)
    b.step(6)
    fb = b.fields()
    for k in fa:
        assert np.array_equal(np.asarray(fa[k]), np.asarray(fb[k])), k
    a.close()
    b.close()


def _columns_lattice(lbm, cols, stream):
    cat = lambda k: np.concatenate([getattr(c, k) for c in cols], axis=-1)
    w0 = cols[0]
    lengths = [c.nx for c in cols]
    lat = lbm.Lattice(1, int(sum(lengths)), 1, 1, w0.molar_mass, w0.D_ref_lat, cat("X0"), cat("T0"), cat("P0"),
                      T_ref=w0.T_ref, bc_lo=w0.bc_lo, bc_hi=w0.bc_hi, inlet_lo_X=w0.inlet_lo_X,
                      inlet_T=w0.inlet_T, col_len=lengths, stream=stream)
    lat.set_porous_field(cat("phi"), cat("tort"), w0.pore_radius)
    lat.set_faradaic_source(cat("faradaic_rate"), 0, 1)
    lat.set_mechanism(w0.mech)
    return lat


@pytest.mark.parametrize("case", ["columns_chemistry", "d2q9_c1"])
def test_graph_step_loop_matches_plain_launches(lbm, case):
    """Replays of the captured step graph, interleaved with plain steps, moment
    reads and synchronisations, give bitwise the plain-launch results after every
    call."""
    import torch
    stream = torch.cuda.Stream()
    if case == "columns_chemistry":
        cols = [synth.config4_column(L, p, i) for L, p, i in zip([30, 45, 17], [0.35, 0.45, 0.3], [0.0, 1.0, 2.0])]
        mk = lambda: _columns_lattice(lbm, cols, stream.cuda_stream)
        G, keys = 4, ("rho_a", "u", "P", "theta", "X", "j_a")
    else:
        w = synth.config1(nx=24, ny=16)
        mk = lambda: lbm.lattice_from_workload(w, stream=stream.cuda_stream)
        G, keys = 2, ("rho_a", "u", "P", "X", "j_a", "rho")
    plain, graph = mk(), mk()
    graph.set_graph(G)
    for n in (1, 8, 3, 9, 4, 2, 12):
        _log(f"{case}: {n} steps")
        plain.step(n)
        graph.step(n)
        fp, fg = plain.fields(), graph.fields()
        for k in keys:
            assert np.array_equal(np.asarray(fp[k]), np.asarray(fg[k])), (case, n, k)
    plain.close()
    graph.close()


def test_health_check_reports_a_non_finite_population(lbm):
    """The conservation / health reduction counts non-finite populations and
    lbm_get_diagnostics returns LBM_EUNSTABLE for them: one population of a snapshot
    is set to NaN on the host and loaded back (a normal load, no kernel sees it before
    the reduction)."""
    w = synth.config1(nx=12, ny=8)
    lat = lbm.lattice_from_workload(w)
    lat.step(3)
    d0 = lat.diagnostics()
    assert d0["rc"] == lbm.LBM_OK and d0["n_nonfinite"] == 0
    blob = bytearray(lat.save())
    L, Q, N = w.M + 1, 9, w.N
    n_rec = 11 * N                                   # node-record planes after the populations
    head = len(blob) - 8 * (L * Q * N + n_rec)
    pops = np.frombuffer(blob, dtype=np.float64, count=L * Q * N, offset=head).copy()
    k = 1 * Q * N + 4 * N + 17                       # species 1, direction 4, node 17
    pops[k] = np.nan
    blob[head:head + 8 * pops.size] = pops.tobytes()
    lat.load(bytes(blob))
    d = lat.diagnostics(check=False)
    lat.close()
    assert d["rc"] == lbm.LBM_EUNSTABLE, d
    assert d["n_nonfinite"] == 1, d


def test_tile_barrier_wait_limit_fails_the_step_loudly(lbm):
    """The D3Q27 species kernel runs two tiles per workgroup, each waiting for its own
    waves at LDS-counter barriers with a bounded wait.  With the bound forced to zero
    from the host every such wait gives up at once: the step must then be reported
    unstable (a NaN population), never hang or pass silently; with the default bound
    the same lattice steps cleanly and matches a fresh run bitwise."""
    w = synth.config3(nx=64, ny=8, nz=4)
    ref = lbm.lattice_from_workload(w)
    ref.step(4)
    good = ref.fields()
    ref.close()
    lat = lbm.lattice_from_workload(w)
    lat.step(2)
    with pytest.raises(lbm.LBMError):
        lat.set_tile_wait_limit(-1)
    lat.set_tile_wait_limit(0)
    lat.step(1)
    d = lat.diagnostics(check=False)
    lat.close()
    _log(f"tile wait limit 0: rc {d['rc']}, non-finite populations {d['n_nonfinite']}")
    assert d["rc"] == lbm.LBM_EUNSTABLE, d
    assert d["n_nonfinite"] > 0, d
    lat = lbm.lattice_from_workload(w)
    lat.set_tile_wait_limit(1 << 18)
    lat.step(4)
    again = lat.fields()
    d = lat.diagnostics(check=False)
    lat.close()
    assert d["rc"] == lbm.LBM_OK, d
    for k in ("rho_a", "u", "P"):
        assert np.array_equal(np.asarray(good[k]), np.asarray(again[k])), k
