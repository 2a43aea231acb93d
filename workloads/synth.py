"""Seeded synthetic workloads for the mean-field reactive porous-media LBM.

This module only produces *inputs*: grid sizes, species molar masses, binary
diffusivities, porosity/tortuosity fields, initial compositions, boundary
descriptions and a synthetic surface mechanism.  It holds none of the
method's arithmetic (no equilibria, no unit system, no relaxation rates);
both the CPU oracle and the GPU path consume the same arrays.

The paper's own workloads (a ternary capillary counter-diffusion run and a
SOFC membrane-electrode assembly, Section 5) need external experimental data
and a Cantera mechanism that are not available, so these seeded stand-ins
reproduce their scales: 1 atm, 1073 K, delta_x = 1 micron (Section 5.2,
Table of parameters), 1-D button-cell columns, porosities 0.3-0.6.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

# Boundary kinds on the x axis (y and z are always periodic).
BC_PERIODIC = 0
BC_BOUNCEBACK = 1
BC_INLET = 2
BC_OUTFLOW = 3

P_ATM = 101325.0

# Lattice kinematic viscosity of the porous 2-D and 3-D workloads with Knudsen diffusion
# (the porous electrode and the porous outflow domain).  At the generic 0.05 the rest state
# of these runs has growing long diagonal waves (the Knudsen force of the species momenta
# feeding the momentum lattice together with the Galilean correction); at 0.3 every mode
# of their domains decays.  1-D columns and the capillary keep 0.05.
KNUDSEN_MULTI_D_NU = 0.3


@dataclass
class Mechanism:
    """Mass-action surface mechanism on one reactive surface.

    Species order inside the stoichiometric tables: M gas species, then K
    surface species (index 0 of the surface block is the vacancy).
    Rates are q_r = kf * prod C^nu_f - kb * prod C^nu_b in mol/(m^2 s), with
    C in mol/m^3 for gas and Gamma*theta in mol/m^2 for surface species, and
    k = A exp(-Ea / (R_U T)).
    """
    K: int
    nu_f: np.ndarray          # (R, M+K) int32 reactant coefficients (= orders)
    nu_b: np.ndarray          # (R, M+K) int32 product coefficients (= orders)
    A_f: np.ndarray           # (R,) SI, mol-based units
    Ea_f: np.ndarray          # (R,) J/mol
    A_b: np.ndarray
    Ea_b: np.ndarray
    gamma: float              # site density, mol/m^2
    a_s: float                # specific surface area, 1/m
    surf_mass: np.ndarray     # (K,) kg/mol
    theta0: np.ndarray        # (K,) initial coverages
    n_sub: int = 4
    n_newton: int = 6
    # adsorbed-phase thermo for the energy lattice, U_k = u_form_k + cv_k T (J/kg);
    # None: no internal energy in the adsorbed phase
    surf_cv: Optional[np.ndarray] = None        # (K,) J/(kg K)
    surf_u_form: Optional[np.ndarray] = None    # (K,) J/kg
    # (R,) 1 for a homogeneous gas-phase reaction (gas species only, zero net mass,
    # q per unit gas volume), 0 for a surface reaction; None: all surface
    homogeneous: Optional[np.ndarray] = None
    # second surface phase (e.g. electrolyte next to electrode): surface_phase (K,) 0/1 assigns
    # each surface species (each phase has its own vacancy); gamma2, a_s2 are that phase's site
    # density and specific area; edge (R,) marks triple-phase-boundary reactions among adsorbed
    # species of both phases, rate per unit edge length, l_tpb edge length per unit volume (1/m^2)
    surface_phase: Optional[np.ndarray] = None
    gamma2: float = 0.0
    a_s2: float = 0.0
    edge: Optional[np.ndarray] = None
    l_tpb: float = 0.0
    # charge transfer (Section 4.1): charge_z (R,) electrons released into the electrode by the
    # forward direction of a TPB edge reaction (0: none), beta_ct (R,) symmetry factors
    charge_z: Optional[np.ndarray] = None
    beta_ct: Optional[np.ndarray] = None

    @property
    def R(self) -> int:
        return int(self.nu_f.shape[0])


@dataclass
class Workload:
    name: str
    lattice: int              # spatial dimension D (1, 2, 3); Q = 3**D
    nx: int
    ny: int
    nz: int
    molar_mass: np.ndarray    # (M,) kg/mol
    D_ref_lat: np.ndarray     # (M,M) binary diffusivities, lattice units at (T_ref, P_ref)
    X0: np.ndarray            # (M,N) initial mole fractions
    P0: np.ndarray            # (N,) initial pressure, Pa
    T0: np.ndarray            # (N,) initial / prescribed temperature, K
    phi: np.ndarray           # (N,) porosity
    tort: np.ndarray          # (N,) tortuosity
    pore_radius: float        # m; <= 0 or inf switches Knudsen diffusion off
    steps: int
    T_ref: float = 1073.0
    P_ref: float = P_ATM
    dx: float = 1.0e-6
    theta_ref: float = 1.0 / 3.0
    nu_lat: float = 0.05
    prandtl: float = 0.7
    energy_on: bool = False
    cv: Optional[np.ndarray] = None       # (M,) J/(kg K)
    u_form: Optional[np.ndarray] = None   # (M,) J/kg  (U_a = u_form + cv*T)
    bc_lo: int = BC_PERIODIC
    bc_hi: int = BC_PERIODIC
    inlet_lo_X: Optional[np.ndarray] = None
    inlet_hi_X: Optional[np.ndarray] = None
    inlet_P: float = P_ATM
    inlet_T: float = 1073.0
    d_visc: int = 0                       # D in 2/D of the stress; 0 -> lattice dimension
    mech: Optional[Mechanism] = None
    faradaic_rate: Optional[np.ndarray] = None   # (N,) mol/(m^3 s) of fuel consumed
    faradaic_species: tuple = (0, 1)             # (fuel, product)
    # electrode coupling (Section 4.2): {"phi_ed": electrode potential V, "omega": (nx,)
    # electrolyte resistivity Ohm m}; None: no charge transport
    electrode: Optional[dict] = None
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.molar_mass.shape[0])

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def Q(self) -> int:
        return 3 ** self.lattice


def synthetic_D_ref(m_gmol: np.ndarray, d0: float = 0.2) -> np.ndarray:
    """Hard-sphere reduced-mass scaling of a synthetic binary diffusivity.

    The (2, 28) g/mol pair receives d0 (lattice units at the reference state).
    """
    m = np.asarray(m_gmol, dtype=np.float64)
    inv = 1.0 / m
    D = d0 * np.sqrt((inv[:, None] + inv[None, :]) / (1.0 / 2.0 + 1.0 / 28.0))
    np.fill_diagonal(D, 0.0)
    return D


def gaussian_random_field(shape, corr_len: float, lo: float, hi: float, seed: int) -> np.ndarray:
    """White noise, spectrally filtered by exp(-k^2 l^2 / 4), affinely mapped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    filt = np.exp(-k2 * corr_len ** 2 / 4.0)
    field_ = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    fmin, fmax = field_.min(), field_.max()
    return lo + (hi - lo) * (field_ - fmin) / (fmax - fmin)


def synthetic_mechanism(m_gas_kg: np.ndarray, seed: int, n_sub: int = 4, n_newton: int = 6) -> Mechanism:
    """10 surface species (vacancy, 5 adsorbates, 4 composites), 20 reversible reactions.

    Reaction families (all site- and mass-balanced):
      5x  G_a + V <-> A_a
      4x  A_i + A_j <-> C_k + V
      8x  G_i + A_j <-> C_k  and  G_j + A_i <-> C_k
      3x  G_i + G_j + V <-> C_k          (for 3 of the 4 composites)
    Pre-factors are drawn log-uniform in [1e2, 1e12] in Cantera's kmol-based
    units and converted to mol-based SI; activation energies uniform in
    [50, 200] kJ/mol.
    """
    rng = np.random.default_rng(seed)
    M = len(m_gas_kg)
    assert M == 5
    K = 10
    S = M + K
    # surface block: 0 = V, 1..5 = A_a, 6..9 = C_k
    pairs = []
    while len(pairs) < 4:
        i, j = sorted(rng.choice(M, size=2, replace=False).tolist())
        if (i, j) not in pairs:
            pairs.append((i, j))
    surf_mass = np.zeros(K)
    surf_mass[0] = 0.0
    surf_mass[1:6] = m_gas_kg
    for k, (i, j) in enumerate(pairs):
        surf_mass[6 + k] = m_gas_kg[i] + m_gas_kg[j]
    gas = lambda a: a
    V = M + 0
    Aa = lambda a: M + 1 + a
    Ck = lambda k: M + 6 + k
    reacs = []
    for a in range(M):
        reacs.append(({gas(a): 1, V: 1}, {Aa(a): 1}))
    for k, (i, j) in enumerate(pairs):
        reacs.append(({Aa(i): 1, Aa(j): 1}, {Ck(k): 1, V: 1}))
    for k, (i, j) in enumerate(pairs):
        reacs.append(({gas(i): 1, Aa(j): 1}, {Ck(k): 1}))
        reacs.append(({gas(j): 1, Aa(i): 1}, {Ck(k): 1}))
    for k, (i, j) in enumerate(pairs[:3]):
        reacs.append(({gas(i): 1, gas(j): 1, V: 1}, {Ck(k): 1}))
    R = len(reacs)
    assert R == 20
    nu_f = np.zeros((R, S), dtype=np.int32)
    nu_b = np.zeros((R, S), dtype=np.int32)
    for r, (lhs, rhs) in enumerate(reacs):
        for s, n in lhs.items():
            nu_f[r, s] = n
        for s, n in rhs.items():
            nu_b[r, s] = n
    logA_f = rng.uniform(2.0, 12.0, R)
    logA_b = rng.uniform(2.0, 12.0, R)
    Ea_f = rng.uniform(50e3, 200e3, R)
    Ea_b = rng.uniform(50e3, 200e3, R)
    order_f = nu_f.sum(axis=1)
    order_b = nu_b.sum(axis=1)
    # kmol-based -> mol-based: rate_mol = 1e3 * A_k * prod (C/1e3)^nu
    A_f = 10.0 ** logA_f * 1e3 ** (1 - order_f)
    A_b = 10.0 ** logA_b * 1e3 ** (1 - order_b)
    theta0 = np.zeros(K)
    theta0[0] = 1.0
    return Mechanism(K=K, nu_f=nu_f, nu_b=nu_b, A_f=A_f, Ea_f=Ea_f, A_b=A_b, Ea_b=Ea_b,
                     gamma=2.6e-5, a_s=1.0e7, surf_mass=surf_mass, theta0=theta0,
                     n_sub=n_sub, n_newton=n_newton)


def _uniform(shape_n, v):
    return np.full(shape_n, float(v))


def config1(nx: int = 64, ny: int = 64, steps: int = 1000, pore_radius: float = 1e-6,
            phi: float = 0.4, tort: float = 3.0) -> Workload:
    """D2Q9 64x64 periodic binary (2, 28 g/mol), isothermal 1073 K, phi 0.4, tau 3,
    r_p 1 micron, x1 = 0.5 + 0.01 sin(2 pi x / 64), u = 0."""
    m = np.array([2.0, 28.0])
    N = nx * ny
    x = np.tile(np.arange(nx), ny)
    x1 = 0.5 + 0.01 * np.sin(2.0 * np.pi * x / 64.0)
    X0 = np.stack([x1, 1.0 - x1])
    return Workload(name="c1_d2q9_periodic_binary", lattice=2, nx=nx, ny=ny, nz=1,
                    molar_mass=m * 1e-3, D_ref_lat=synthetic_D_ref(m), X0=X0,
                    P0=_uniform(N, P_ATM), T0=_uniform(N, 1073.0), phi=_uniform(N, phi),
                    tort=_uniform(N, tort), pore_radius=pore_radius, steps=steps, T_ref=1073.0)


def config2(kn_index: int = 0, nx: int = 1024, ny: int = 64, steps: int = 20000) -> Workload:
    """D2Q9 counter-diffusion capillary: x1 = 1 inlet at x=0, x1 = 0 inlet at x=nx-1,
    equal pressure, phi 0.5, tau 1, energy on, Kn = 0.01 * 10^(3k/7)."""
    m = np.array([2.0, 28.0])
    N = nx * ny
    x = np.tile(np.arange(nx), ny)
    x1 = 1.0 - x / (nx - 1.0)
    X0 = np.stack([x1, 1.0 - x1])
    D = synthetic_D_ref(m)
    kn = 0.01 * 10.0 ** (3.0 * kn_index / 7.0)
    m_kg = m * 1e-3
    R_U = 8.314462618
    # lattice thermal speed of the lightest species at T_ref: sqrt(theta_ref)
    # D^k_1 = D_12 / Kn; D^k = (d0 / 3 dx) sqrt(8 R1T / pi)  (phi = tau = 1 in Kn def)
    Dk1 = D[0, 1] / kn
    d0 = 3.0 * Dk1 / np.sqrt(8.0 * (1.0 / 3.0) / np.pi)   # in units of dx
    rp = 0.5 * d0 * 1e-6
    cv = 2.5 * R_U / m_kg
    return Workload(name=f"c2_d2q9_capillary_kn{kn_index}", lattice=2, nx=nx, ny=ny, nz=1,
                    molar_mass=m_kg, D_ref_lat=D, X0=X0, P0=_uniform(N, P_ATM),
                    T0=_uniform(N, 1073.0), phi=_uniform(N, 0.5), tort=_uniform(N, 1.0),
                    pore_radius=rp, steps=steps, T_ref=1073.0, energy_on=True, cv=cv,
                    u_form=np.zeros(2), bc_lo=BC_INLET, bc_hi=BC_INLET,
                    inlet_lo_X=np.array([1.0, 0.0]), inlet_hi_X=np.array([0.0, 1.0]),
                    inlet_P=P_ATM, inlet_T=1073.0, meta={"kn": kn})


def config3_species(seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(2.0, 44.0, 5))


def config3(nx: int = 256, ny: int = 128, nz: int = 128, steps: int = 2000, seed: int = 3,
            n_sub: int = 1, n_newton: int = 2, with_mech: bool = True) -> Workload:
    """D3Q27 porous electrode: 5 species, GRF porosity (corr. length 8) in [0.3, 0.6],
    tortuosity phi^-1/2, r_p 1 micron, T linear 973 -> 1073 K along x, 10 surface
    species / 20 reactions, X0 = 0.2 each, u = 0, 1 atm."""
    m = config3_species(seed)
    m_kg = m * 1e-3
    shape = (nz, ny, nx)
    phi = gaussian_random_field(shape, 8.0, 0.3, 0.6, seed + 100).reshape(-1)
    N = nx * ny * nz
    x = np.tile(np.arange(nx), ny * nz)
    T = 973.0 + 100.0 * x / max(nx - 1, 1)
    X0 = np.full((5, N), 0.2)
    mech = synthetic_mechanism(m_kg, seed + 200, n_sub=n_sub, n_newton=n_newton) if with_mech else None
    return Workload(name="c3_d3q27_porous_electrode", lattice=3, nx=nx, ny=ny, nz=nz,
                    molar_mass=m_kg, D_ref_lat=synthetic_D_ref(m), X0=X0,
                    P0=_uniform(N, P_ATM), T0=T, phi=phi, tort=phi ** -0.5,
                    pore_radius=1e-6, steps=steps, T_ref=1073.0, mech=mech,
                    nu_lat=KNUDSEN_MULTI_D_NU)


def config3_energy(nx: int = 10, ny: int = 6, nz: int = 4, seed: int = 3) -> Workload:
    """C3 physics with the energy lattice on (a unit-test case, not a benchmark):
    gas cv_a = (5/2) R_U / m_a, u_form 0; adsorbates with the same molar heat
    capacity (cv_k = (5/2) R_U / m_k) and a formation energy of -20 kJ/mol for
    the composites, so adsorption moves internal energy between the phases."""
    R_U = 8.314462618
    w = config3(nx=nx, ny=ny, nz=nz, seed=seed)
    m = np.asarray(w.molar_mass)
    sm = np.asarray(w.mech.surf_mass)
    with np.errstate(divide="ignore"):
        scv = np.where(sm > 0, 2.5 * R_U / np.where(sm > 0, sm, 1.0), 0.0)
    suf = np.zeros_like(sm)
    suf[6:] = -2.0e4 / sm[6:]
    mech = replace(w.mech, surf_cv=scv, surf_u_form=suf)
    return replace(w, name="c3_energy_reactive", energy_on=True, cv=2.5 * R_U / m, u_form=np.zeros(len(m)),
                   mech=mech)


def homogeneous_dimerisation(nx: int = 8, ny: int = 1, phi: float = 0.4, kf: float = 2.0e6,
                             kb: float = 5.0e7, x_a: float = 0.9, with_surface: bool = False) -> Workload:
    """Binary gas 2A <=> B (m_B = 2 m_A: zero net mass) as a homogeneous gas-phase
    reaction with temperature-independent rate constants (kf in m^3/(mol s), kb in
    1/s), uniform state, isothermal 1073 K, D1Q3 (ny = 1) or D2Q9, periodic.  The
    mechanism carries an inert two-species surface (vacancy only) because the
    chemistry solve always has coverages.  with_surface adds the surface reaction
    A + V <=> A(s) next to the homogeneous one."""
    m = np.array([14.0, 28.0])
    lattice = 1 if ny == 1 else 2
    N = nx * ny
    X0 = np.stack([_uniform(N, x_a), _uniform(N, 1.0 - x_a)])
    nu_f = [[2, 0, 0, 0]]
    nu_b = [[0, 1, 0, 0]]
    A_f, A_b, hom = [kf], [kb], [1]
    if with_surface:                      # A + V <=> A(s), mol/(m^2 s) per (mol/m^3) (mol/m^2)
        nu_f.append([1, 0, 1, 0])
        nu_b.append([0, 0, 0, 1])
        A_f.append(2.0e4)
        A_b.append(1.0e5)
        hom.append(0)
    R = len(A_f)
    mech = Mechanism(K=2, nu_f=np.array(nu_f, dtype=np.int32), nu_b=np.array(nu_b, dtype=np.int32),
                     A_f=np.array(A_f), Ea_f=np.zeros(R), A_b=np.array(A_b), Ea_b=np.zeros(R),
                     gamma=2.6e-5, a_s=1.0e7, surf_mass=np.array([0.0, 0.014]), theta0=np.array([1.0, 0.0]),
                     n_sub=1, n_newton=3, homogeneous=np.array(hom, dtype=np.int32))
    return Workload(name="homogeneous_dimerisation", lattice=lattice, nx=nx, ny=ny, nz=1,
                    molar_mass=m * 1e-3, D_ref_lat=synthetic_D_ref(m), X0=X0,
                    P0=_uniform(N, P_ATM), T0=_uniform(N, 1073.0), phi=_uniform(N, phi),
                    tort=_uniform(N, phi ** -0.5), pore_radius=1e-6, steps=100, T_ref=1073.0, mech=mech)


def two_phase_tpb(nx: int = 6, ny: int = 4, phi: float = 0.4, theta_a1: float = 0.5,
                  with_gas: bool = True, kf: float = 3.0e7, kb: float = 1.0e7) -> Workload:
    """Two surface phases with a triple-phase-boundary edge reaction, 3 inert-ish gas
    species (2, 18, 28 g/mol), isothermal 1073 K, D2Q9 periodic, uniform state.
    Surface species: V1, A1 (phase 1: Gamma 2.6e-5, a_s 1e7), V2, A2 (phase 2:
    Gamma 1.3e-5, a_s 5e6); edge reaction A1 + V2 <=> A2 + V1 (kf, kb in
    m^2 mol^-1 s^-1 per unit edge length, l_tpb 2e12 m^-2).  with_gas adds the
    adsorption G1 + V1 <=> A1 on phase 1 and the desorption A2 <=> G1 + V2 on
    phase 2 (A carries the mass of G1, 18 g/mol)."""
    m = np.array([2.0, 18.0, 28.0])
    N = nx * ny
    X0 = np.stack([_uniform(N, 0.3), _uniform(N, 0.3), _uniform(N, 0.4)])
    M = 3
    # columns: G0 G1 G2 | V1 A1 V2 A2
    nu_f = [[0, 0, 0, 0, 1, 1, 0]]
    nu_b = [[0, 0, 0, 1, 0, 0, 1]]
    A_f, A_b, edge = [kf], [kb], [1]
    if with_gas:
        nu_f += [[0, 1, 0, 1, 0, 0, 0], [0, 0, 0, 0, 0, 0, 1]]
        nu_b += [[0, 0, 0, 0, 1, 0, 0], [0, 1, 0, 0, 0, 1, 0]]
        A_f += [2.0e4, 3.0e6]
        A_b += [1.0e5, 4.0e4]
        edge += [0, 0]
    R = len(A_f)
    mech = Mechanism(K=4, nu_f=np.array(nu_f, dtype=np.int32), nu_b=np.array(nu_b, dtype=np.int32),
                     A_f=np.array(A_f), Ea_f=np.zeros(R), A_b=np.array(A_b), Ea_b=np.zeros(R),
                     gamma=2.6e-5, a_s=1.0e7, surf_mass=np.array([0.0, 0.018, 0.0, 0.018]),
                     theta0=np.array([1.0 - theta_a1, theta_a1, 1.0, 0.0]), n_sub=1, n_newton=3,
                     surface_phase=np.array([0, 0, 1, 1], dtype=np.int32), gamma2=1.3e-5, a_s2=5.0e6,
                     edge=np.array(edge, dtype=np.int32), l_tpb=2.0e12)
    return Workload(name="two_phase_tpb", lattice=2, nx=nx, ny=ny, nz=1, molar_mass=m * 1e-3,
                    D_ref_lat=synthetic_D_ref(m), X0=X0, P0=_uniform(N, P_ATM), T0=_uniform(N, 1073.0),
                    phi=_uniform(N, phi), tort=_uniform(N, phi ** -0.5), pore_radius=1e-6, steps=100,
                    T_ref=1073.0, mech=mech)


def electrode_slab(nx: int = 12, ny: int = 2, phi_ed: float = 0.05, omega: float = 5.0e-3,
                   beta: float = 0.5, with_gas: bool = True, kf: float = 3.0e3,
                   kb: float = 1.0e3, phi: float = 0.4, lattice: int = 2,
                   energy: bool = False) -> Workload:
    """The two-phase TPB mechanism of two_phase_tpb with its edge reaction as a
    charge transfer (A1 + V2 <=> A2 + V1 + e-, one electron into the electrode,
    symmetry factor beta), on a D2Q9 slab periodic in y and bounce-back at both
    x ends; electrode potential phi_ed (V) and a uniform electrolyte resistivity
    omega (Ohm m) along x.  lattice=1 with ny=1 gives the same cell as a D1Q3 column.
    energy turns the energy lattice on (gas cv_a = (5/2) R_U / m_a, u_form 0, no
    adsorbed-phase thermo), so the electrical energy source acts on the temperature."""
    w = two_phase_tpb(nx=nx, ny=ny, phi=phi, with_gas=with_gas, kf=kf, kb=kb)
    w.lattice = lattice
    if energy:
        m = np.asarray(w.molar_mass)
        w.energy_on = True
        w.cv = 2.5 * 8.314462618 / m
        w.u_form = np.zeros(len(m))
    R = w.mech.R
    z = np.zeros(R, dtype=np.int32)
    z[0] = 1
    w.mech.charge_z = z
    w.mech.beta_ct = np.full(R, beta)
    w.bc_lo = BC_BOUNCEBACK
    w.bc_hi = BC_BOUNCEBACK
    w.electrode = {"phi_ed": float(phi_ed), "omega": np.full(nx, float(omega))}
    w.name = "electrode_slab"
    return w


def config4_columns(seed: int = 4, n_cols: int = 64, lmin: int = 200, lmax: int = 2000):
    rng = np.random.default_rng(seed)
    lengths = rng.integers(lmin, lmax + 1, n_cols)
    phis = rng.uniform(0.3, 0.5, n_cols)
    currents = 2.0 * np.arange(n_cols) / max(n_cols - 1, 1)     # A/cm^2
    return lengths, phis, currents


def config4_electrode_cells(seed: int = 4):
    """The 64 ragged c4 column lengths and porosities as closed D1Q3 electrode cells
    (electrode_slab with slow kinetics kf 3e-2, kb 1e-2, resistivity 1e-3 Ohm m, initial
    electrode potential 0.3 V), each with a target area current density: c4's currents,
    at least 0.1 A/cm^2, in A/m^2.  Returns (cells, targets)."""
    lengths, phis, currents = config4_columns(seed)
    cells = [electrode_slab(nx=int(L), ny=1, phi=float(p_), lattice=1, kf=3.0e-2, kb=1.0e-2,
                            omega=1.0e-3, phi_ed=0.3) for L, p_ in zip(lengths, phis)]
    targets = np.maximum(np.asarray(currents, dtype=np.float64), 0.1) * 1.0e4
    return cells, targets


def config4_column(length: int, phi: float, current_A_cm2: float, seed: int = 4,
                   steps: int = 50000, n_sub: int = 1, n_newton: int = 2,
                   n_util: int = 2, delta_util: float = 2e-6) -> Workload:
    """One D1Q3 button-cell anode column: inlet (0.97, 0.03, 0, 0, 0) at x=0, bounce-back
    at x=L-1, Faradaic fuel->product source over the last n_util nodes, isothermal 1073.15 K."""
    m = config3_species(3)
    m_kg = m * 1e-3
    N = int(length)
    Xin = np.array([0.97, 0.03, 0.0, 0.0, 0.0])
    X0 = np.repeat(Xin[:, None], N, axis=1)
    F = 96485.33212
    i_SI = current_A_cm2 * 1e4
    rate = np.zeros(N)
    rate[N - n_util:] = i_SI / (2.0 * F * delta_util)
    mech = synthetic_mechanism(m_kg, 3 + 200, n_sub=n_sub, n_newton=n_newton)
    return Workload(name="c4_d1q3_column", lattice=1, nx=N, ny=1, nz=1, molar_mass=m_kg,
                    D_ref_lat=synthetic_D_ref(m), X0=X0, P0=_uniform(N, P_ATM),
                    T0=_uniform(N, 1073.15), phi=_uniform(N, phi), tort=_uniform(N, phi ** -0.5),
                    pore_radius=1e-6, steps=steps, T_ref=1073.15, bc_lo=BC_INLET,
                    bc_hi=BC_BOUNCEBACK, inlet_lo_X=Xin, inlet_P=P_ATM, inlet_T=1073.15,
                    d_visc=3, mech=mech, faradaic_rate=rate,
                    meta={"current_A_cm2": current_A_cm2})


def config5(nx: int = 1024, ny: int = 256, steps: int = 2000, seed: int = 5,
            porosity: str = "grf") -> Workload:
    """D2Q9 1024x256, 3 species (2, 18, 28), GRF porosity [0.3, 0.6] (porosity="grf") or
    uniform 0.45 (porosity="uniform"), tortuosity phi^-1/2, r_p 1 micron, 1073 K;
    inlet X=(0.8,0.1,0.1) at x=0, outflow at x=nx-1, X0 linear."""
    m = np.array([2.0, 18.0, 28.0])
    m_kg = m * 1e-3
    if porosity == "uniform":
        phi = np.full(nx * ny, 0.45)
    else:
        phi = gaussian_random_field((ny, nx), 8.0, 0.3, 0.6, seed + 100).reshape(-1)
    N = nx * ny
    x = np.tile(np.arange(nx), ny)
    s = x / max(nx - 1, 1)
    Xin = np.array([0.8, 0.1, 0.1])
    Xout = np.array([0.1, 0.45, 0.45])
    X0 = Xin[:, None] * (1.0 - s)[None, :] + Xout[:, None] * s[None, :]
    return Workload(name="c5_d2q9_porous_outflow", lattice=2, nx=nx, ny=ny, nz=1,
                    molar_mass=m_kg, D_ref_lat=synthetic_D_ref(m), X0=X0,
                    P0=_uniform(N, P_ATM), T0=_uniform(N, 1073.0), phi=phi, tort=phi ** -0.5,
                    pore_radius=1e-6, steps=steps, T_ref=1073.0, bc_lo=BC_INLET,
                    bc_hi=BC_OUTFLOW, inlet_lo_X=Xin, inlet_P=P_ATM, inlet_T=1073.0,
                    nu_lat=KNUDSEN_MULTI_D_NU)


def with_sizes(w: Workload, **kw) -> Workload:
    return replace(w, **kw)
