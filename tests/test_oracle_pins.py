"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with an
independent statement (stated moments, conservation laws, a linearised
continuum model built from the kinetic equation's coefficients, exact
symmetries, lattice marginalisation, textbook lattice weights).
"""
import math
import os
from dataclasses import replace
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import lbm_oracle as lo
from workloads import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rng(seed=0):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# Lattice / product form
# --------------------------------------------------------------------------

def test_d3q27_weights_golden():
    """Product form at (xi=0, P=1/3) gives the textbook D3Q27 weights."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "d3q27_weights.txt"))
            if l.strip() and not l.startswith("#")]
    ref = {int(a): float(b) for a, b in rows}
    c = lo.lattice_velocities(3)
    w = lo.lattice_weights(c)
    for i in range(27):
        nnz = int(np.count_nonzero(c[i]))
        assert abs(w[i] - ref[nnz]) < 1e-15
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("D", [1, 2, 3])
def test_species_equilibrium_moments(D):
    """eq 27eq: sum f^eq = phi rho_a, sum f^eq c = rho_a u, sum f^eq c c = phi rho_a (v v + R_a T I)."""
    r = _rng(D)
    n = 50
    c = lo.lattice_velocities(D)
    phi = r.uniform(0.3, 1.0, n)
    rho = r.uniform(0.5, 3.0, n)
    RaT = r.uniform(0.02, 0.3, n)
    v = r.uniform(-0.1, 0.1, (D, n))
    f = lo.species_equilibrium(c, phi * rho, v, RaT)
    assert np.allclose(f.sum(0), phi * rho, rtol=1e-14, atol=0)
    for a in range(D):
        m1 = (f * c[:, a, None]).sum(0)
        assert np.allclose(m1, rho * phi * v[a], rtol=1e-13, atol=1e-16)
        for b in range(D):
            m2 = (f * (c[:, a] * c[:, b])[:, None]).sum(0)
            exp = phi * rho * (v[a] * v[b] + (RaT if a == b else 0.0))
            assert np.allclose(m2, exp, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_energy_equilibrium_moments(D):
    """eqs g0momTotalEnergy, geq1mom, geq2mom: zeroth phi rho E, first (H + u^2/2phi^2) rho u,
    second (H + u^2/2phi^2) P^eq + (P/phi) u u, with P^eq = phi rho v v + phi P I (eq Peq)."""
    r = _rng(10 + D)
    n = 40
    c = lo.lattice_velocities(D)
    phi = r.uniform(0.3, 1.0, n)
    rho = r.uniform(0.5, 3.0, n)
    RT = r.uniform(0.02, 0.3, n)
    U = r.uniform(0.1, 2.0, n)
    u = r.uniform(-0.05, 0.05, (D, n))
    v = u / phi
    g = lo.energy_equilibrium(c, phi * rho, U, RT, v)
    u2 = (u * u).sum(0)
    E = U + u2 / (2 * phi ** 2)
    H = U + RT
    P = rho * RT
    assert np.allclose(g.sum(0), phi * rho * E, rtol=1e-13)
    for a in range(D):
        q = (g * c[:, a, None]).sum(0)
        assert np.allclose(q, (H + u2 / (2 * phi ** 2)) * rho * u[a], rtol=1e-12, atol=1e-15)
        for b in range(D):
            R = (g * (c[:, a] * c[:, b])[:, None]).sum(0)
            Peq = phi * rho * (u[a] / phi) * (u[b] / phi) + (phi * P if a == b else 0.0)
            exp = (H + u2 / (2 * phi ** 2)) * Peq + (P / phi) * u[a] * u[b]
            assert np.allclose(R, exp, rtol=1e-12, atol=1e-15)


def test_reaction_population_moments():
    """eqs Dotfr, m1fDotc: the source population carries rho_dot and rho_dot u / phi."""
    r = _rng(3)
    c = lo.lattice_velocities(3)
    n = 30
    phi = r.uniform(0.3, 1.0, n)
    u = r.uniform(-0.05, 0.05, (3, n))
    RaT = r.uniform(0.02, 0.3, n)
    rdot = r.normal(size=n)
    fr = rdot * lo.product_form(c, u / phi, (u / phi) ** 2 + RaT)
    assert np.allclose(fr.sum(0), rdot, rtol=1e-13, atol=1e-15)
    for a in range(3):
        assert np.allclose((fr * c[:, a, None]).sum(0), rdot * u[a] / phi, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------
# Conservation (eq finalNumericalEquationsReactive, eq f)
# --------------------------------------------------------------------------

def test_conservation_without_drag():
    w = synth.config1(nx=32, ny=16, pore_radius=float("inf"))
    o = lo.Oracle(w)
    m0 = o.fa.sum(axis=(1, 2))
    M0 = o.f.sum()
    scale = (o.f.sum(0) * np.sqrt(o.macro()["RT"])).sum()
    o.step(300)
    assert np.all(np.abs(o.fa.sum(axis=(1, 2)) - m0) / m0 < 1e-13)
    assert abs(o.f.sum() - M0) / M0 < 1e-13
    j = np.array([(o.f * o.c[:, d, None]).sum() for d in range(2)])
    assert np.all(np.abs(j) / scale < 1e-13)


def test_momentum_change_equals_knudsen_force():
    """With the Knudsen drag on, the mixture momentum changes by exactly sum_x F^k per step."""
    w = synth.config1(nx=32, ny=16)
    o = lo.Oracle(w)
    o.step(20)
    for _ in range(5):
        mac = o.macro()
        j0 = mac["j"].sum(axis=1)
        Fk = mac["Fk"].sum(axis=1)
        o.step(1)
        j1 = o.macro()["j"].sum(axis=1)
        scale = np.abs(mac["Fk"]).sum() + 1e-300
        assert np.all(np.abs((j1 - j0) - Fk) / scale < 1e-11)


# --------------------------------------------------------------------------
# Hydrodynamic limit (eqs dtrhoa, constit2; Appendix A)
# --------------------------------------------------------------------------

def _x1_mode(o, nx):
    X = o.moments()["X"][0].reshape(-1, nx).mean(axis=0)
    return np.fft.fft(X)[1] / (nx / 2)


def test_binary_diffusion_decay_matches_D12():
    """Knudsen off: the first Fourier mode of x_1 decays at D_12 k^2 (from eqs dtrhoa and
    constit2 linearised at uniform pressure).  Diffusivity reduced 20x so the diffusive
    mode separates from the acoustic and viscous ones."""
    scale = 0.05
    w = synth.config1(nx=64, ny=1, pore_radius=float("inf"))
    w = replace(w, D_ref_lat=w.D_ref_lat * scale)
    o = lo.Oracle(w)
    ts, amps = [], []
    o.step(1000)
    for _ in range(10):
        o.step(500)
        ts.append(o.step_count)
        amps.append(abs(_x1_mode(o, 64)))
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    k = 2 * math.pi / 64
    D12 = 0.2 * scale    # synthetic binary diffusivity of the (2, 28) pair at the reference state
    assert abs(rate / (D12 * k * k) - 1.0) < 3e-3


def _dgm_linear_prediction(m, X, D12, Dk, phi, k, RaT, ts):
    """Linearised continuum dusty-gas model written from the kinetic equation's
    coefficients (eq stefanMaxwell): friction P X_a X_b / D_ab, Knudsen drag P X_a / D^k_a,
    partial pressure phi rho_a R_a T, continuity phi d rho_a/dt + div(rho_a u_a) = 0."""
    from scipy.linalg import expm
    rho_a = X * 1.0 / RaT          # P = 1 in pressure units
    P = (rho_a * RaT).sum()
    A = np.zeros((4, 4), complex)
    A[0, 2] = -1j * k / phi
    A[1, 3] = -1j * k / phi
    A[2, 0] = -1j * k * phi * RaT[0]
    A[3, 1] = -1j * k * phi * RaT[1]
    K12 = P * X[0] * X[1] / D12
    # d(rho_a u_a)/dt += K12 (u_b - u_a) - P X_a / D^k_a u_a
    A[2, 2] = -K12 / rho_a[0] - P * X[0] / Dk[0] / rho_a[0]
    A[2, 3] = K12 / rho_a[1]
    A[3, 3] = -K12 / rho_a[1] - P * X[1] / Dk[1] / rho_a[1]
    A[3, 2] = K12 / rho_a[0]
    x0 = np.array([0.01 / RaT[0], -0.01 / RaT[1], 0, 0], complex)   # isobaric x_1 perturbation
    out = []
    for t in ts:
        s = expm(A * t) @ x0
        cbar = rho_a / m
        cp = s[:2] / m
        out.append((cp[0] - X[0] * cp.sum()) / cbar.sum())
    return np.array(out)


def test_knudsen_decay_matches_linear_dusty_gas_model():
    scale = 0.05
    w = synth.config1(nx=64, ny=1, pore_radius=1e-6 * scale)
    w = replace(w, D_ref_lat=w.D_ref_lat * scale)
    o = lo.Oracle(w)
    m = np.array([2.0, 28.0])
    RaT = (1.0 / 3.0) * 2.0 / m
    phi, tort = 0.4, 3.0
    Dk = (phi / tort) * (2e-6 * scale / (3 * 1e-6)) * np.sqrt(8 * RaT / math.pi)   # Section 5.1, d_0 = 2 r_p
    ts, amps = [], []
    for _ in range(8):
        o.step(500)
        ts.append(o.step_count)
        amps.append(_x1_mode(o, 64))
    pred = _dgm_linear_prediction(m, np.array([0.5, 0.5]), 0.2 * scale, Dk, phi, 2 * math.pi / 64, RaT, ts)
    ratio = np.abs(np.array(amps)) / np.abs(pred)
    assert np.all(np.abs(ratio - 1.0) < 2e-3), ratio


# --------------------------------------------------------------------------
# Porosity placement: exact mean-field symmetry f(phi) = phi f(1)
# --------------------------------------------------------------------------

def _periodic_energy_workload(nx=16, ny=8, phi=1.0, seed=0):
    r = _rng(seed)
    w = synth.config2(nx=nx, ny=ny)
    N = nx * ny
    x1 = 0.5 + 0.05 * r.standard_normal(N)
    T0 = 1073.0 * (1.0 + 0.02 * r.standard_normal(N))
    P0 = synth.P_ATM * (1.0 + 0.01 * r.standard_normal(N))
    return replace(w, bc_lo=synth.BC_PERIODIC, bc_hi=synth.BC_PERIODIC, pore_radius=float("inf"),
                   X0=np.stack([x1, 1 - x1]), T0=T0, P0=P0, phi=np.full(N, phi))


def test_porosity_scaling_symmetry_isothermal():
    """Knudsen off, uniform phi: every phi-placement in the equilibria, the Galilean
    correction and the extended velocity makes populations scale exactly as phi * f(phi=1)."""
    base = synth.config1(nx=16, ny=8, pore_radius=float("inf"))
    r = _rng(1)
    x1 = 0.5 + 0.05 * r.standard_normal(base.N)
    base = replace(base, X0=np.stack([x1, 1 - x1]), P0=synth.P_ATM * (1 + 0.01 * r.standard_normal(base.N)))
    o1 = lo.Oracle(replace(base, phi=np.full(base.N, 1.0)))
    o2 = lo.Oracle(replace(base, phi=np.full(base.N, 0.4)))
    o1.step(60)
    o2.step(60)
    assert np.max(np.abs(o2.fa - 0.4 * o1.fa)) / np.max(np.abs(o1.fa)) < 1e-13
    assert np.max(np.abs(o2.f - 0.4 * o1.f)) / np.max(np.abs(o1.f)) < 1e-13
    assert np.max(np.abs(o2.macro()["u"] - 0.4 * o1.macro()["u"])) < 1e-13 * np.max(np.abs(o1.macro()["u"])) + 1e-20


def test_porosity_scaling_symmetry_energy():
    o1 = lo.Oracle(_periodic_energy_workload(phi=1.0))
    o2 = lo.Oracle(_periodic_energy_workload(phi=0.5))
    o1.step(40)
    o2.step(40)
    for a, b in ((o2.fa, o1.fa), (o2.f, o1.f), (o2.g, o1.g)):
        assert np.max(np.abs(a - 0.5 * b)) / np.max(np.abs(b)) < 1e-12


# --------------------------------------------------------------------------
# Lattice reduction: the product form marginalises (Section 2.2)
# --------------------------------------------------------------------------

def _marginal(pop, c_hi, D_lo):
    """Sum populations of the higher lattice over the last velocity component."""
    Q_lo = 3 ** D_lo
    out = np.zeros(pop.shape[:-2] + (Q_lo,) + pop.shape[-1:])
    for i in range(c_hi.shape[0]):
        i_lo = sum((c_hi[i, a] + 1) * 3 ** a for a in range(D_lo))
        out[..., i_lo, :] += pop[..., i, :]
    return out


def test_d2q9_y_uniform_reduces_to_d1q3_with_energy():
    nx = 24
    w2 = _periodic_energy_workload(nx=nx, ny=3, phi=0.45, seed=4)
    # make every y-row identical
    for arr in ("X0", "T0", "P0", "phi"):
        a = getattr(w2, arr)
        a = a.reshape(a.shape[:-1] + (3, nx))
        a[..., :, :] = a[..., :1, :]
    w2 = replace(w2, pore_radius=1e-6, tort=np.full(w2.N, 2.0))
    w1 = replace(w2, lattice=1, ny=1, X0=w2.X0[:, :nx], T0=w2.T0[:nx], P0=w2.P0[:nx],
                 phi=w2.phi[:nx], tort=w2.tort[:nx])
    o2, o1 = lo.Oracle(w2), lo.Oracle(w1)
    o2.step(50)
    o1.step(50)
    for p2, p1 in ((o2.fa, o1.fa), (o2.f, o1.f), (o2.g, o1.g)):
        mg = _marginal(p2, o2.c, 1)[..., :nx]
        assert np.max(np.abs(mg - p1)) / np.max(np.abs(p1)) < 1e-13


def test_d3q27_z_uniform_reduces_to_d2q9():
    w2 = synth.config1(nx=12, ny=6)
    r = _rng(7)
    x1 = 0.5 + 0.05 * r.standard_normal(w2.N)
    phi = r.uniform(0.3, 0.6, w2.N)
    w2 = replace(w2, X0=np.stack([x1, 1 - x1]), phi=phi, tort=phi ** -0.5)
    rep = lambda a: np.concatenate([a, a], axis=-1)
    w3 = replace(w2, lattice=3, nz=2, X0=rep(w2.X0), P0=rep(w2.P0), T0=rep(w2.T0), phi=rep(w2.phi),
                 tort=rep(w2.tort))
    o3, o2 = lo.Oracle(w3), lo.Oracle(w2)
    o3.step(40)
    o2.step(40)
    for p3, p2 in ((o3.fa, o2.fa), (o3.f, o2.f)):
        mg = _marginal(p3, o3.c, 2)[..., :w2.N]
        assert np.max(np.abs(mg - p2)) / np.max(np.abs(p2)) < 1e-13


# --------------------------------------------------------------------------
# Species velocity system (eqs transform1, stefanMaxwell)
# --------------------------------------------------------------------------

def test_species_solve_equals_paper_system_without_knudsen():
    """R4 reduces to the printed V-form system when 1/tau^k = 0."""
    w = synth.config5(nx=24, ny=6)
    w = replace(w, pore_radius=float("inf"), bc_lo=0, bc_hi=0)
    o = lo.Oracle(w)
    o.step(30)
    mac = o.macro()
    M = o.M
    for n in range(0, o.N, 7):
        A = np.zeros((M, M))
        for a in range(M):
            A[a, a] = 1.0 + 0.5 * mac["inv_tau_a"][a, n]
            for b in range(M):
                if b != a:
                    A[a, b] = -0.5 * mac["inv_tau_ab"][a, b, n] * mac["Y"][b, n]
        for d in range(2):
            rhs = mac["jt"][:, d, n] / mac["rho_a"][:, n] - mac["u"][d, n]
            V = np.linalg.solve(A, rhs)
            assert np.allclose(V, mac["Va"][:, d, n], rtol=1e-10, atol=1e-16)


def test_lb_momentum_is_trapezoidal_shift_of_kinetic_momentum():
    """The LB first moment equals rho_a u_a - 1/2 (first moment of the kinetic collision
    term of eq stefanMaxwell), with the kinetic coefficients P X_a X_b / D_ab and
    P X_a / D^k_a taken straight from the paper (Knudsen on, 3 species), P X_a being the
    partial pressure rho_a R_a T of Section 2.1."""
    w = synth.config5(nx=24, ny=6)
    w = replace(w, bc_lo=0, bc_hi=0)
    o = lo.Oracle(w)
    o.step(30)
    mac = o.macro()
    M, D = o.M, 2
    X, T = mac["X"], mac["T"]
    RaT = mac["RaT"]
    Pa = mac["rho_a"] * RaT                        # Dalton partial pressures
    P = Pa.sum(0)
    Dab = w.D_ref_lat[:, :, None] * ((T / w.T_ref) ** 1.5 / P)[None, None, :]
    Dk = (o.phi / o.tort)[None, :] * (2 * w.pore_radius / (3 * w.dx)) * np.sqrt(8 * RaT / math.pi)
    for d in range(D):
        for a in range(M):
            ua = mac["ja"][a, d] / mac["rho_a"][a]
            om = -Pa[a] / Dk[a] * ua
            for b in range(M):
                if b != a:
                    ub = mac["ja"][b, d] / mac["rho_a"][b]
                    om = om + Pa[a] * X[b] / Dab[a, b] * (ub - ua)
            lhs = mac["jt"][a, d]
            rhs = mac["ja"][a, d] - 0.5 * om
            assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-14 * np.abs(mac["ja"]).max())


# --------------------------------------------------------------------------
# Surface chemistry (Section 4 with reading R13)
# --------------------------------------------------------------------------

def _chem_oracle(steps=3):
    w = synth.config4_column(length=12, phi=0.4, current_A_cm2=0.0, n_sub=2, n_newton=4)
    w = replace(w, faradaic_rate=None)
    o = lo.Oracle(w)
    o.step(steps)
    return o


def test_chemistry_conserves_sites_and_mass():
    o = _chem_oracle()
    mac = o.macro()
    src, th = o.chemistry(mac)
    mech = o.mech
    assert np.all(np.abs(th.sum(0) - 1.0) < 1e-13)
    gas = (src * o.rho_unit).sum(0)                                          # kg/m^3 total volume
    surf = mech.a_s * mech.gamma * ((th - o.theta) * mech.surf_mass[:, None]).sum(0)
    scale = (o.phi * mac["rho_a"].sum(0)) * o.rho_unit
    assert np.all(np.abs(gas + surf) / scale < 1e-13)
    assert np.any(np.abs(gas) / scale > 1e-8)          # chemistry actually did something


def test_coverages_stay_valid_over_run():
    o = _chem_oracle(steps=25)
    assert np.all(np.abs(o.theta.sum(0) - 1.0) < 1e-12)
    assert np.all(o.theta > -1e-12)


def test_langmuir_isotherm():
    """One reaction G + V <-> A(s) with the gas held fixed reaches
    theta_A = K c / (1 + K c), K = kf / kb."""
    m = np.array([0.002, 0.028])
    nu_f = np.array([[1, 0, 1, 0]], dtype=np.int32)
    nu_b = np.array([[0, 0, 0, 1]], dtype=np.int32)
    mech = synth.Mechanism(K=2, nu_f=nu_f, nu_b=nu_b, A_f=np.array([3e11]), Ea_f=np.array([60e3]),
                           A_b=np.array([2e14]), Ea_b=np.array([90e3]), gamma=2.6e-5, a_s=1e7,
                           surf_mass=np.array([0.0, 0.002]), theta0=np.array([1.0, 0.0]),
                           n_sub=2, n_newton=5)
    N = 4
    w = synth.Workload(name="langmuir", lattice=1, nx=N, ny=1, nz=1, molar_mass=m,
                       D_ref_lat=synth.synthetic_D_ref(np.array([2.0, 28.0])),
                       X0=np.array([[0.3] * N, [0.7] * N]), P0=np.full(N, synth.P_ATM),
                       T0=np.full(N, 1073.0), phi=np.full(N, 0.5), tort=np.ones(N),
                       pore_radius=float("inf"), steps=1, mech=mech)
    o = lo.Oracle(w)
    mac = o.macro()
    for _ in range(400):
        src, th = o.chemistry(mac)
        o.theta = th                      # gas composition held at its initial value
    c = mac["rho_a"][0] * o.rho_unit / m[0]
    R_U = 8.314462618
    K = (3e11 * math.exp(-60e3 / (R_U * 1073.0))) / (2e14 * math.exp(-90e3 / (R_U * 1073.0)))
    theta_A = K * c / (1 + K * c)
    assert np.allclose(o.theta[1], theta_A, rtol=1e-10)


# --------------------------------------------------------------------------
# Energy lattice: isobaric thermal decay (eqs dtE, qneq, lambda)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("x1", [1.0, 0.5])
def test_thermal_decay_matches_thermal_diffusivity(x1):
    """An isobaric temperature sine decays at alpha k^2 with alpha = lambda/(rho C_p)
    = (1/omega_1 - 1/2) R T = nu / Pr, independent of the composition."""
    nx = 64
    x = np.arange(nx)
    w = synth.config2(nx=nx, ny=1)
    X = np.array([x1, 1.0 - x1])
    w = replace(w, bc_lo=synth.BC_PERIODIC, bc_hi=synth.BC_PERIODIC, pore_radius=float("inf"),
                X0=np.repeat(X[:, None], nx, axis=1), T0=1073.0 * (1 + 0.01 * np.sin(2 * np.pi * x / nx)),
                P0=np.full(nx, synth.P_ATM))
    o = lo.Oracle(w)
    ts, amps = [], []
    o.step(200)
    for _ in range(6):
        o.step(100)
        ts.append(o.step_count)
        amps.append(abs(np.fft.fft(o.moments()["T"])[1]))
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    k = 2 * math.pi / nx
    alpha = w.nu_lat / w.prandtl
    assert abs(rate / (alpha * k * k) - 1.0) < 0.03


def test_energy_density_unit_against_si():
    """The lattice energy density unit is rho_unit c^2 (Section 5.2 unit system,
    R16): the energy lattice's initial zeroth moment at rest, times rho_unit c^2,
    equals the SI internal energy density phi sum_a c_a m_a (u_form_a + cv_a T)
    with c_a = X_a P / (R_U T) of the ideal-gas inputs."""
    w = synth.config3_energy(nx=6, ny=4, nz=3)
    o = lo.Oracle(w)
    T = np.asarray(w.T0)
    c_a = np.asarray(w.X0) * np.asarray(w.P0)[None, :] / (lo.R_U * T[None, :])          # mol/m^3
    m = np.asarray(w.molar_mass)
    U_si = (c_a * m[:, None] * (np.asarray(w.u_form)[:, None] + np.asarray(w.cv)[:, None] * T[None, :])).sum(axis=0)
    got = o.g.sum(axis=0) * o.rho_unit * o.c2
    assert np.allclose(got, np.asarray(w.phi) * U_si, rtol=1e-13, atol=0.0)


def test_unified_internal_energy_kept_through_chemistry():
    """Eqs temperatureCell, InternalEnergyCell_PC, g0mom_source and g_source:
    without electrical sources the unified internal energy (fluid + adsorbed
    phase at one T) is unchanged by the chemistry, so over one step from rest
    (v = 0, periodic, the collision and the stream keep sum g) the fluid's
    energy total changes by minus the adsorbed phase's change, both at the
    step's temperature.  A dropped or sign-flipped source term fails."""
    w = synth.config3_energy(nx=6, ny=4, nz=3)
    o = lo.Oracle(w)
    T1 = o.macro()["T"]
    es0 = o.surface_energy(o.theta, T1).sum()
    g0 = o.g.sum()
    o.step(1)
    des = o.surface_energy(o.theta, T1).sum() - es0
    dg = o.g.sum() - g0
    assert abs(des) > 1e-6 * abs(g0)                       # the adsorbed phase really took energy
    assert abs(dg + des) <= 1e-9 * abs(des), (dg, des)


def test_homogeneous_reaction_reaches_mass_action_equilibrium():
    """Homogeneous 2A <=> B (eqs sumRhoDot, totalFluidReactionRate): the
    implicit chemistry's fixed point is the mass-action equilibrium
    c_B / c_A^2 = kf / kb, and the mixture mass is unchanged (m_B = 2 m_A)."""
    w = synth.homogeneous_dimerisation()
    o = lo.Oracle(w)
    rho0 = o.macro()["rho_a"].sum(axis=0)
    o.step(1000)
    mac = o.macro()
    cA = mac["rho_a"][0] * o.rho_unit / o.m[0]
    cB = mac["rho_a"][1] * o.rho_unit / o.m[1]
    ratio = w.mech.A_f[0] / w.mech.A_b[0]
    assert np.allclose(cB / cA ** 2, ratio, rtol=1e-10, atol=0.0)
    assert np.allclose(mac["rho_a"].sum(axis=0), rho0, rtol=1e-12, atol=0.0)


def test_homogeneous_reaction_rate_is_per_gas_volume():
    """One step with slow kinetics: dc_A = -2 (kf c_A^2 - kb c_B) dt, the gas
    concentration changes at the mass-action rate itself (eq dtrhoa: phi rho_a
    balances a source per unit total volume = phi times the per-gas-volume
    rate), independent of the porosity and of the surface area a_s."""
    for phi in (0.3, 0.8):
        w = synth.homogeneous_dimerisation(phi=phi, kf=2.0e2, kb=5.0e3)
        o = lo.Oracle(w)
        mac = o.macro()
        cA = mac["rho_a"][0] * o.rho_unit / o.m[0]
        cB = mac["rho_a"][1] * o.rho_unit / o.m[1]
        expect = -2.0 * (w.mech.A_f[0] * cA ** 2 - w.mech.A_b[0] * cB) * o.dt
        o.step(1)
        cA1 = o.macro()["rho_a"][0] * o.rho_unit / o.m[0]
        assert np.allclose(cA1 - cA, expect, rtol=1e-5, atol=0.0), (cA1 - cA, expect)


def test_two_phase_edge_reaction_equilibrium_and_balances():
    """Two surface phases joined by a TPB edge reaction A1 + V2 <=> A2 + V1 (eqs
    totalSurfaceReactionRate, totalSurfaceReactionRateTPB_electrode/_electrolyte):
    the implicit update's fixed point is the mass-action equilibrium
    theta_A2 theta_V1 / (theta_A1 theta_V2) = kf / kb, each phase keeps its sites,
    and the adsorbate moles per volume a1 G1 theta_A1 + a2 G2 theta_A2 are kept."""
    w = synth.two_phase_tpb(nx=3, ny=3, with_gas=False)
    o = lo.Oracle(w)
    m = w.mech
    held0 = m.a_s * m.gamma * o.theta[1] + m.a_s2 * m.gamma2 * o.theta[3]
    o.step(400)
    th = o.theta
    assert np.allclose(th[0] + th[1], 1.0, rtol=0, atol=1e-13)
    assert np.allclose(th[2] + th[3], 1.0, rtol=0, atol=1e-13)
    assert np.allclose(m.a_s * m.gamma * th[1] + m.a_s2 * m.gamma2 * th[3], held0, rtol=1e-12, atol=0)
    assert np.allclose(th[3] * th[0] / (th[1] * th[2]), m.A_f[0] / m.A_b[0], rtol=1e-9, atol=0)


def test_two_phase_edge_rate_scaled_by_tpb_length_over_area():
    """One step with slow kinetics: each phase's coverage changes at the edge rate
    times l_TPB / (a^(s) Gamma) of its own surface (eq totalSurfaceReactionRate)."""
    w = synth.two_phase_tpb(nx=2, ny=2, with_gas=False, kf=3.0e1, kb=1.0e1)
    o = lo.Oracle(w)
    m = w.mech
    th = o.theta
    C = np.array([m.gamma * th[0], m.gamma * th[1], m.gamma2 * th[2], m.gamma2 * th[3]])
    q = m.A_f[0] * C[1] * C[2] - m.A_b[0] * C[3] * C[0]                  # per unit edge length
    o.step(1)
    d1 = o.theta[1] - th[1]
    d2 = o.theta[3] - th[3]
    assert np.allclose(d1, -m.l_tpb / (m.a_s * m.gamma) * q * o.dt, rtol=1e-5, atol=0)
    assert np.allclose(d2, m.l_tpb / (m.a_s2 * m.gamma2) * q * o.dt, rtol=1e-5, atol=0)


def test_two_phase_chemistry_conserves_sites_and_mass():
    """With gas adsorption on phase 1, the edge transfer and desorption from phase 2:
    sites per phase and gas + both adsorbed phases' mass are conserved per node."""
    w = synth.two_phase_tpb(nx=3, ny=2, with_gas=True)
    o = lo.Oracle(w)
    mac = o.macro()
    src, th = o.chemistry(mac)
    m = w.mech
    assert np.all(np.abs(th[0] + th[1] - 1.0) < 1e-13) and np.all(np.abs(th[2] + th[3] - 1.0) < 1e-13)
    gas = (src * o.rho_unit).sum(0)
    a_k = np.array([m.a_s, m.a_s, m.a_s2, m.a_s2])
    g_k = np.array([m.gamma, m.gamma, m.gamma2, m.gamma2])
    surf = ((a_k * g_k * m.surf_mass)[:, None] * (th - o.theta)).sum(0)
    scale = (o.phi * mac["rho_a"].sum(0)) * o.rho_unit
    assert np.all(np.abs(gas + surf) / scale < 1e-13)
    assert np.any(np.abs(gas) / scale > 1e-8)


# --------------------------------------------------------------------------
# Charge transfer and charge transport (Sections 4.1-4.2, R30)
# --------------------------------------------------------------------------

def _charge_slab(theta0, z=1, beta=0.5, kf=3.0e1, kb=1.0e1, nx=3, ny=2, phi_ed=0.0, omega=0.0):
    w = synth.electrode_slab(nx=nx, ny=ny, phi_ed=phi_ed, omega=omega, beta=beta, with_gas=False,
                             kf=kf, kb=kb)
    w.mech.theta0 = np.asarray(theta0, dtype=np.float64)
    w.mech.charge_z = np.array([z], dtype=np.int32)
    return w


def test_charge_transfer_rests_at_the_nernst_potential():
    """The net charge-transfer rate vanishes where the electrode potential balances the
    mass-action quotient: dPhi_eq = (R_U T / (z F)) ln(kb C_A2 C_V1 / (kf C_A1 C_V2)); there
    the step produces no current and leaves the coverages unchanged, while 20 mV above it
    the oxidation runs (positive current)."""
    th0 = [0.4, 0.6, 0.7, 0.3]
    w = _charge_slab(th0, z=2, beta=0.3)
    m = w.mech
    C = np.array([m.gamma * th0[0], m.gamma * th0[1], m.gamma2 * th0[2], m.gamma2 * th0[3]])
    T = w.T0[0]
    eq = lo.R_U * T / (2 * lo.F_C) * math.log(m.A_b[0] * C[3] * C[0] / (m.A_f[0] * C[1] * C[2]))
    w.electrode["phi_ed"] = eq
    o = lo.Oracle(w)
    o.step(1)
    w2 = _charge_slab(th0, z=2, beta=0.3, phi_ed=eq + 0.02)
    o2 = lo.Oracle(w2)
    o2.step(1)
    assert np.all(o2.i_v > 1e6)
    assert np.all(np.abs(o.i_v) < 1e-9 * o2.i_v)
    assert np.allclose(o.theta, np.asarray(th0)[:, None], rtol=0, atol=1e-15)


def test_charge_transfer_tafel_slope_is_beta_z_f_over_rt():
    """Far from equilibrium (no product on the surface, slow kinetics) the oxidation current
    grows as exp(beta z F dPhi / (R_U T)): raising the potential by 10 mV multiplies it by
    exp(beta z F 0.01 / (R_U T)), with beta = 0.3, z = 2 (not 1 - beta, not z = 1)."""
    th0 = [0.4, 0.6, 1.0, 0.0]
    cur = []
    for ph in (0.05, 0.06):
        o = lo.Oracle(_charge_slab(th0, z=2, beta=0.3, phi_ed=ph))
        o.step(1)
        cur.append(o.i_v.copy())
    T = 1073.0
    ratio = math.exp(0.3 * 2 * lo.F_C * 0.01 / (lo.R_U * T))
    assert np.allclose(cur[1] / cur[0], ratio, rtol=1e-6, atol=0)


def test_charge_balance_current_equals_transferred_adsorbate():
    """eq volumetricCurrent against the coverage bookkeeping: the charge one step releases per
    unit volume, I^(v) dt, is z F times the moles of A2 formed on the electrolyte surface,
    a2 Gamma2 (theta_A2' - theta_A2), with z = 2."""
    th0 = [0.4, 0.6, 0.9, 0.1]
    w = _charge_slab(th0, z=2, beta=0.5, kf=3.0e5, kb=1.0e5, phi_ed=0.03)
    o = lo.Oracle(w)
    m = w.mech
    o.step(1)
    moles = m.a_s2 * m.gamma2 * (o.theta[3] - th0[3])
    assert np.all(moles > 0)
    assert np.allclose(o.i_v * o.dt, 2 * lo.F_C * moles, rtol=1e-9, atol=0)


def test_charge_transport_closed_form_for_uniform_current():
    """eqs areaCurrentDensity, electrolytePotential with a uniform volumetric current I and
    resistivity Omega, integrated from x = 0 cell by cell: I^(a)(x_i) = (i + 1) I dx and
    Phi(x_i) = Omega I dx^2 (i + 1)(i + 2) / 2 on every (y) line."""
    w = synth.electrode_slab(nx=7, ny=3, omega=0.25)
    o = lo.Oracle(w)
    I = 3.0e9
    ia, pel = o.charge_transport(np.full(o.N, I))
    i = np.tile(np.arange(w.nx), w.ny).astype(np.float64)
    dx = w.dx
    assert np.allclose(ia, (i + 1) * I * dx, rtol=1e-13, atol=0)
    assert np.allclose(pel, 0.25 * I * dx * dx * (i + 1) * (i + 2) / 2, rtol=1e-13, atol=0)


def test_electrical_energy_source_enters_the_energy_total():
    """R31 with eqs InternalEnergyCell_PC, g0mom_source, g_source: over one step from rest
    (bounce-back ends and periodic y keep sum g, no adsorbed-phase thermo, no gas
    reaction) the energy lattice total changes by exactly the electrical source: minus
    the electrical work |dPhi| I^(v) dt when the electrolyte has no resistance, and the
    ohmic heat (a_electrolyte / l_TPB) I^(v)^2 Omega dx dt on top when it has one, both
    rebuilt here from the step's current (the charge balance pins I^(v))."""
    for omega in (0.0, 40.0):
        w = synth.electrode_slab(nx=8, ny=2, energy=True, with_gas=False, omega=omega, phi_ed=0.05)
        o = lo.Oracle(w)
        g0 = o.g.sum()
        dphi = o.dphi.copy()
        o.step(1)
        iv = o.i_v
        m = w.mech
        work = np.abs(dphi) * iv * o.dt
        heat = (m.a_s2 / m.l_tpb) * iv ** 2 * omega * w.dx * o.dt
        expect = (heat - work).sum() / (o.rho_unit * o.c2)
        dg = o.g.sum() - g0
        assert np.all(iv > 0)
        assert abs(dg - expect) <= 1e-9 * abs(expect), (omega, dg, expect)
        if omega == 0.0:
            assert dg < 0                                         # work leaves the fluid
        else:
            assert heat.sum() > work.sum() and dg > 0             # ohmic heating wins here


def test_current_control_reaches_the_target_on_every_line():
    """R32 (Section 4.2): with a target area current density per x line, every step's end
    current I^(a)(x = nx - 1) equals the target to rounding, and the line asked for the
    larger current runs at the higher electrode potential (oxidation current grows with
    the potential)."""
    w = synth.electrode_slab(nx=12, ny=2, omega=5e-3)
    target = np.array([1.0e6, 1.6e6])
    w.electrode["target_ia"] = target
    w.electrode["n_secant"] = 6
    o = lo.Oracle(w)
    for _ in range(4):
        o.step(1)
        assert np.allclose(o.i_a[o.line_end], target, rtol=1e-12, atol=0)
        assert o.ped[1] > o.ped[0]


def test_faradaic_source_moves_the_prescribed_moles():
    """R26 against a mole balance: in a periodic D1Q3 column (streaming and collision keep
    every species' total), one step changes the fuel total by minus and the product total by
    plus sum_n rate_n dt moles (per unit lattice volume), the other species not at all."""
    w = synth.config4_column(40, 0.4, 1.5)
    w = replace(w, bc_lo=synth.BC_PERIODIC, bc_hi=synth.BC_PERIODIC, mech=None, inlet_lo_X=None)
    o = lo.Oracle(w)
    before = o.fa.sum(axis=(1, 2))
    o.step(1)
    moles = (o.fa.sum(axis=(1, 2)) - before) * o.rho_unit / o.m
    fu, pr = w.faradaic_species
    expect = np.asarray(w.faradaic_rate).sum() * o.dt
    assert expect > 0
    assert abs(moles[fu] + expect) <= 1e-9 * expect and abs(moles[pr] - expect) <= 1e-9 * expect
    others = [a for a in range(w.M) if a not in (fu, pr)]
    assert np.all(np.abs(moles[others]) <= 1e-12 * expect)


def test_inlet_and_outflow_keep_a_matching_rest_state():
    """R17, R18 on rest states: with the whole domain at the inlet's composition, pressure and
    temperature and at rest, an inlet at x = 0 and an outflow at x = nx - 1 (porosity 0.45)
    leave every field unchanged for 30 steps (the inlet equilibrium at the node's zero
    velocity equals the state it replaces: a wrong composition, pressure, temperature or
    porosity factor there fails)."""
    w = synth.config5(nx=24, ny=4, steps=10, porosity="uniform")
    N = w.N
    X = np.repeat(np.asarray(w.inlet_lo_X)[:, None], N, axis=1)
    w = replace(w, X0=X, P0=np.full(N, w.inlet_P), T0=np.full(N, w.inlet_T))
    assert w.bc_lo == synth.BC_INLET and w.bc_hi == synth.BC_OUTFLOW
    o = lo.Oracle(w)
    m0 = o.moments()
    o.step(30)
    m1 = o.moments()
    for k in ("rho_a", "P", "X"):
        assert np.max(np.abs(np.asarray(m1[k]) - np.asarray(m0[k]))) <= 1e-13 * np.max(np.abs(m0[k])), k
    assert np.max(np.abs(m1["u"])) <= 1e-15


def test_inlet_and_outflow_keep_a_matching_uniform_flow():
    """R17, R18 with velocity: the domain at the inlet's composition, pressure and temperature,
    every lattice at its equilibrium moving with u = 0.02 along x (Knudsen off, uniform
    porosity, so a periodic domain would keep it), an inlet at x = 0 and an outflow at
    x = nx - 1: 30 steps change nothing.  An inlet equilibrium at rest instead of the node's
    velocity, or an outflow that copies another direction, fails."""
    w = synth.config5(nx=24, ny=4, steps=10, porosity="uniform")
    N = w.N
    X = np.repeat(np.asarray(w.inlet_lo_X)[:, None], N, axis=1)
    w = replace(w, X0=X, P0=np.full(N, w.inlet_P), T0=np.full(N, w.inlet_T), pore_radius=float("inf"))
    o = lo.Oracle(w)
    RaT = o.RaT(o.T_field)
    rho_a = X * (w.P0 / w.P_ref)[None, :] / RaT
    v = [np.full(N, 0.02 / o.phi[0]), np.zeros(N)]
    o.fa = np.stack([o.species_eq(o.phi * rho_a[a], v, RaT[a]) for a in range(o.M)])
    Y, _, _ = o.composition(rho_a)
    RT = (Y * RaT).sum(axis=0)
    o.f = (o.phi * rho_a.sum(axis=0)) * lo.product_form(o.c, v, [RT + v[d] ** 2 for d in range(o.D)])
    m0 = o.moments()
    o.step(30)
    m1 = o.moments()
    for k in ("rho_a", "P", "X", "u", "j_a"):
        assert np.max(np.abs(np.asarray(m1[k]) - np.asarray(m0[k]))) <= 1e-13 * np.max(np.abs(m0[k])), k


def test_absent_species_changes_nothing():
    """R19 by marginalisation: a third species with zero density everywhere (18 g/mol, not the
    lightest, so the unit system is unchanged) stays at zero and leaves the binary run of
    the other two unchanged, Knudsen drag on, 20 steps, to 1e-13 (an unguarded division by
    rho_a = 0 gives NaN; a nonzero quasi-equilibrium for it moves mass)."""
    w2 = synth.config1(nx=16, ny=4)
    m3 = np.array([2.0, 28.0, 18.0])
    D3 = synth.synthetic_D_ref(m3)
    D3[:2, :2] = w2.D_ref_lat
    w3 = replace(w2, molar_mass=m3 * 1e-3, D_ref_lat=D3, X0=np.vstack([w2.X0, np.zeros(w2.N)]))
    a, b = lo.Oracle(w2), lo.Oracle(w3)
    a.step(20)
    b.step(20)
    ma, mb = a.moments(), b.moments()
    for k in ("rho_a", "j_a"):
        ra, rb = np.asarray(ma[k]), np.asarray(mb[k])
        assert np.max(np.abs(rb[:2] - ra)) <= 1e-13 * np.max(np.abs(ra)), k
        assert np.all(rb[2] == 0.0), k
    for k in ("u", "P"):
        assert np.max(np.abs(np.asarray(mb[k]) - np.asarray(ma[k]))) <= 1e-13 * max(np.max(np.abs(ma[k])), 1e-3), k


def test_temperature_of_a_moving_mixture():
    """R7 with the energy equilibrium's pinned zeroth moment phi rho (U + v^2/2): a uniform
    binary mixture moving at u = (0.03, -0.01) in porosity 0.4 (v = u / phi), every lattice at
    its moving equilibrium at 1073 K, periodic, Knudsen off: the temperature read back from
    the energy lattice is 1073 K at the start and after 5 steps (1e-12), and the flow keeps
    its velocity.  Reading the kinetic energy with u instead of v = u / phi fails."""
    R_U = lo.R_U
    w = synth.config1(nx=8, ny=4, pore_radius=float("inf"))
    N = w.N
    m = np.asarray(w.molar_mass)
    X = np.stack([np.full(N, 0.5), np.full(N, 0.5)])
    w = replace(w, X0=X, energy_on=True, cv=2.5 * R_U / m, u_form=np.zeros(2))
    o = lo.Oracle(w)
    RaT = o.RaT(o.T_field)
    rho_a = X * (w.P0 / w.P_ref)[None, :] / RaT
    u = (0.03, -0.01)
    v = [np.full(N, u[0] / o.phi[0]), np.full(N, u[1] / o.phi[0])]
    o.fa = np.stack([o.species_eq(o.phi * rho_a[a], v, RaT[a]) for a in range(o.M)])
    Y, _, _ = o.composition(rho_a)
    RT = (Y * RaT).sum(axis=0)
    rho = rho_a.sum(axis=0)
    o.f = (o.phi * rho) * lo.product_form(o.c, v, [RT + v[d] ** 2 for d in range(o.D)])
    U = (Y * (o.uf_lat[:, None] + o.cv_lat[:, None] * o.T_field[None, :])).sum(axis=0)
    o.g = o.g_equilibrium(o.phi * rho, U, RT, v)
    assert np.allclose(o.macro()["T"], 1073.0, rtol=1e-12, atol=0)
    o.step(5)
    assert np.allclose(o.macro()["T"], 1073.0, rtol=1e-12, atol=0)
    mu = np.asarray(o.moments()["u"])
    assert np.allclose(mu[0], u[0], rtol=1e-12, atol=0) and np.allclose(mu[1], u[1], rtol=1e-12, atol=0)


def test_gradient_of_linear_fields_with_mirror_ends():
    """R9 on closed forms: for A = 2x (D2Q9, bounce-back x ends, periodic y) the isotropic
    gradient 3 sum_i w_i c_i A(x + c_i) is exactly (2, 0) at interior nodes (sum_i w_i c_i c_i
    = I/3); at the x ends the ghost A(x + c) := A(x) halves the x component to 1 (the three
    outward directions see no difference); the y component stays 0 everywhere."""
    nx, ny = 7, 5
    w = replace(synth.config1(nx=nx, ny=ny), bc_lo=synth.BC_BOUNCEBACK, bc_hi=synth.BC_BOUNCEBACK)
    o = lo.Oracle(w)
    x = np.tile(np.arange(nx), ny).astype(np.float64)
    A = 2.0 * x
    gx, gy = o.gradient(A, 0), o.gradient(A, 1)
    ends = (x == 0) | (x == nx - 1)
    assert np.allclose(gx[~ends], 2.0, rtol=0, atol=1e-13)
    assert np.allclose(gx[ends], 1.0, rtol=0, atol=1e-13)
    assert np.allclose(gy, 0.0, rtol=0, atol=1e-13)


def test_varying_porosity_rests_at_uniform_phi_p():
    """R20 (porosity applied pointwise): the model's pressure tensor is phi P I, so a binary
    mixture at rest in a porosity varying along x (0.4 +- 0.1) is in equilibrium when phi P
    is uniform (P = P0 0.4 / phi): 20 steps keep every velocity below 1e-15, while the same
    porosity with uniform P starts a flow (|u| > 1e-3)."""
    nx, ny = 16, 4
    w = synth.config1(nx=nx, ny=ny)
    x = np.tile(np.arange(nx), ny)
    phi = 0.4 + 0.1 * np.sin(2 * np.pi * x / nx)
    X = np.stack([np.full(w.N, 0.5), np.full(w.N, 0.5)])
    out = {}
    for label, P in (("phiP", 101325.0 * 0.4 / phi), ("P", np.full(w.N, 101325.0))):
        o = lo.Oracle(replace(w, phi=phi, P0=P, X0=X))
        o.step(20)
        m = o.moments()
        out[label] = max(np.max(np.abs(m["u"])), np.max(np.abs(m["j_a"])))
    assert out["phiP"] < 1e-15 and out["P"] > 1e-3, out


def test_momentum_lattice_takes_the_reaction_mass_exactly():
    """R24 (the momentum lattice's own rho in the mass-source ratio): C3 physics periodic, after
    5 steps the momentum-lattice density has drifted from sum rho_a by several percent (weak
    coupling), yet one more step changes the momentum lattice's total by exactly the step's
    reaction source sum src (1e-9 of it); with the species density in the ratio it would
    change by src rho / sum rho_a."""
    w = synth.config3(nx=6, ny=4, nz=3)
    o = lo.Oracle(w)
    o.step(5)
    mac = o.macro()
    assert np.max(np.abs(mac["rho"] - mac["rho_a"].sum(0)) / mac["rho"]) > 1e-2
    src, _ = o.chemistry(mac)                 # the step's own source (the call changes no state)
    f0 = o.f.sum()
    o.step(1)
    assert abs(src.sum()) > 1e-4
    assert abs((o.f.sum() - f0) - src.sum()) <= 1e-9 * abs(src.sum())
