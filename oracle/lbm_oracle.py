"""Plain FP64 CPU oracle of the mean-field reactive porous-media lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP library: it re-derives every formula from the paper (Sawant & Karlin,
"Mean field lattice Boltzmann model for reactive mixtures in porous media").

Everything is numpy float64, vectorised over nodes but otherwise written stage
by stage in the paper's order and notation.  Lattice units: delta_x = delta_t = 1.

Readings adopted where the paper is silent, garbled or self-inconsistent
(each one is referenced where it is used):

  R1  tau_ab = D_ab m_a m_b / (m R_U T)  (the printed expression is inverted;
      this is the coefficient P X_a X_b / (D_ab rho_a) = Y_b / tau_ab of the
      kinetic equation, Section 2.1).
  R2  tau^k_a = D^k_a m_a / (R_U T)  (same inversion).
  R3  f*_a uses xi = u_a / phi, P = R_a T + xi^2 (the species quasi-equilibrium
      of Section 2.2; first moment rho_a u_a).
  R4  the second-order species velocities solve
        (1 + 1/2tau_a + 1/2tau^k_a) j_a - sum_{b!=a} Y_a/(2 tau_ab) j_b = j~_a,
      obtained by re-deriving the trapezoidal transform with the Knudsen term;
      equal to the printed system whenever 1/tau^k = 0 or u = 0.
  R5  species equilibria use the momentum-lattice velocity u = j / rho.
  R6  u^ex = u + F^k / (omega rho)  (the printed product form is dimensionally
      inconsistent; the additive shift injects exactly F^k per step).
  R7  temperature from E - v^2/2 with v = u/phi (consistent with E = U + u^2/(2 phi^2)).
  R8  energy equilibrium operator O_a A = RT dA/dv_a + v_a A, v = u/phi.
  R9  isotropic gradient d_a A(x) = 3 sum_i w_i c_ia A(x + c_i); mirror ghost
      A(x + c_i) := A(x) across non-periodic boundaries.
  R10 gradients use time-t fields.
  R11 natural bulk viscosity: the bracket [-s + mu(2/D - R/C_v)] is zero.
  R12 D1Q3 / D2Q9 are the product form with the missing directions dropped.
  R13 surface chemistry: backward Euler on (gas, surface) over n_sub sub-steps
      with n_newton Newton iterations each (dense LU with partial pivoting, no
      early exit), then an extent-based conservative update.
  R14 D_ab = D_ab^ref (T/T_ref)^{3/2} (P_ref/P_s) with the species (Dalton)
      pressure P_s = sum_a rho_a R_a T; constant nu and Pr.  With this, the
      kinetic coefficients P X_a X_b / D_ab read P X_a as the partial pressure
      rho_a R_a T of Section 2.1, so the species lattices do not depend on the
      momentum-lattice density (which drifts from sum_a rho_a under weak coupling).
  R15 constant specific heats, U_a = u_form_a + cv_a T.
  R16 lattice units: theta_ref = R_lightest T_ref = 1/3, pressure unit P_ref,
      density unit P_ref / c^2, c^2 = R_U T_ref / (m_min theta_ref).
  R17 inlet: missing populations := equilibrium of the inlet state moving with
      the boundary node's velocity at the time level being streamed.  For the
      energy lattice the inlet fixes the temperature of what enters: its missing
      populations are the equilibrium at the inlet temperature of the node's own
      mixture (momentum-lattice density and composition at that time level).
  R18 outflow: missing populations copied from the upstream neighbour.
  R19 rho_a = 0: f*_a := 0, u_a := u.
  R21 D^k_a = (phi/tau) (d_0/3) sqrt(8 R_U T / (pi m_a)), d_0 = 2 r_p.
  R24 momentum-lattice rho in P, f^ex and the mass-source ratio.
  R25 the diffusion velocities in the interdiffusion energy flux are taken
      relative to the species mass-average velocity, V_a = u_a - sum_b Y_b u_b,
      so that sum_a rho_a V_a = 0 holds exactly (in the continuum limit this is
      u_a - u; on the lattice the momentum-lattice u drifts from the species'
      barycentric velocity, and a nearly pure species is almost collisionless).
  R26 Faradaic source: fuel consumed / product produced at a prescribed
      volumetric molar rate (explicit).
  R30 charge transfer (Section 4.1, eq volumetricCurrent; the rate law is not
      printed): a TPB edge reaction that releases z electrons into the
      electrode has k_f exp(beta z F dPhi / (R_U T)) and
      k_b exp(-(1 - beta) z F dPhi / (R_U T)), dPhi = Phi_electrode -
      Phi_electrolyte, beta the symmetry factor (mass action with a
      Butler-Volmer potential factor).  I^(v) = F l_TPB sum_r z_r xi_r / dt with
      the step's extents.  Charge transport (eqs areaCurrentDensity,
      electrolytePotential) integrates along x with the rectangle rule over the
      cells 0..x of each (y, z) line, Phi_electrolyte = 0 before cell 0; a
      step's rates take the potentials integrated from the previous step's
      currents (dPhi = Phi_electrode before the first step).
  R31 electrical energy source (Section 4.1, eqs for P_elec, P_Omega, U_source):
      the printed U_source = (-P_Omega + P_elec) dt has both signs reversed
      against the text that defines the terms (electrical work leaves the
      fluid, ohmic heat enters it); taken as U_source = (P_Omega - P_elec) dt
      with P_elec = |dPhi| I^(v), P_Omega = (a_electrolyte / l_TPB) I^(v)^2
      Omega dx, a_electrolyte the specific area of the second surface phase,
      dPhi and I^(v) those of the step's chemistry.  It enters the unified
      internal energy before the adsorbed phases are subtracted (eq
      InternalEnergyCell_PC), so only with the energy lattice on.
  R32 current control (Section 4.2, the secant on the electrode potential): with
      a target area current density per x line, each step first varies the
      line's electrode potential so that I^(a) at the line's last node, from
      this step's chemistry at the step's electrolyte potential, equals the
      target: secant iterates start at the line's present potential and 10 mV
      above it, a fixed number of updates, none where the two last currents
      are equal; the step then runs at the last iterate.

Pins: tests/test_oracle_pins.py, tests/test_oracle_pins_flow.py and
tests/test_oracle_tangent.py check this code against statements independent of it
(conservation, closed forms, equilibria, continuum models and linear-wave rates,
Graham's law, marginalisation, mole and charge balances, finite differences).
Parity unpinned (no pin of their own, covered by the GPU parity tests only): R5, R10,
the momentum-lattice rho of R24 in P and f^ex (its use in the mass-source ratio is
pinned), and which upstream node the outflow of R18 copies from.
"""
from __future__ import annotations

import math

import numpy as np

R_U = 8.314462618       # J/(mol K)
F_C = 96485.33212       # C/mol

# x-axis boundary kinds (y and z are periodic)
BC_PERIODIC = 0
BC_BOUNCEBACK = 1
BC_INLET = 2
BC_OUTFLOW = 3


# ---------------------------------------------------------------------------
# Section 2.2: standard lattice and the product form
# ---------------------------------------------------------------------------

def lattice_velocities(D: int) -> np.ndarray:
    """c_i with components in {-1, 0, 1}; i = sum_a (c_ia + 1) 3^a (x fastest)."""
    Q = 3 ** D
    c = np.zeros((Q, D), dtype=np.int64)
    for i in range(Q):
        for a in range(D):
            c[i, a] = (i // 3 ** a) % 3 - 1
    return c


def psi(ci: int, xi, P):
    """Psi_0 = 1 - P, Psi_{+1} = (xi + P)/2, Psi_{-1} = (-xi + P)/2."""
    if ci == 0:
        return 1.0 - P
    if ci == 1:
        return 0.5 * (xi + P)
    return 0.5 * (-xi + P)


def product_form(c: np.ndarray, xi, P) -> np.ndarray:
    """Psi_i = prod_a Psi_{c_ia}(xi_a, P_aa); xi, P indexable by direction a."""
    Q, D = c.shape
    out = []
    for i in range(Q):
        v = None
        for a in range(D):
            t = psi(int(c[i, a]), xi[a], P[a])
            v = t if v is None else v * t
        out.append(v)
    return np.stack(out)


def lattice_weights(c: np.ndarray) -> np.ndarray:
    """w_i = product form at zero velocity and P = 1/3."""
    D = c.shape[1]
    return product_form(c, [0.0] * D, [1.0 / 3.0] * D)


def species_equilibrium(c, phi_rho_a, v, RaT):
    """f^eq_a = phi rho_a prod_a Psi(v_a, v_a^2 + R_a T), v = u/phi  (eq 27eq)."""
    D = c.shape[1]
    P = [v[d] ** 2 + RaT for d in range(D)]
    return phi_rho_a * product_form(c, [v[d] for d in range(D)], P)


def energy_equilibrium(c, phi_rho, U, RT, v):
    """Energy equilibrium g^eq = phi rho prod Psi(O_a, O_a^2) E  (eq geq_i with reading R8).

    With O_a = RT d/dv_a + v_a and E = U + sum v_a^2 / 2 the operator acts per
    direction:  O^0 1 = 1,  O 1 = v,  O^2 1 = RT + v^2,
                O (v^2/2) = RT v + v^3/2,  O^2 (v^2/2) = RT^2 + 5/2 RT v^2 + v^4/2.
    """
    Q, D = c.shape
    a = []
    e = []
    for d in range(D):
        vd = v[d]
        xi1 = vd
        P1 = RT + vd * vd
        xiE = RT * vd + 0.5 * vd ** 3
        PE = RT * RT + 2.5 * RT * vd * vd + 0.5 * vd ** 4
        a.append({0: 1.0 - P1, 1: 0.5 * (xi1 + P1), -1: 0.5 * (-xi1 + P1)})
        e.append({0: 0.5 * vd * vd - PE, 1: 0.5 * (xiE + PE), -1: 0.5 * (-xiE + PE)})
    out = []
    for i in range(Q):
        prod_a = None
        for d in range(D):
            t = a[d][int(c[i, d])]
            prod_a = t if prod_a is None else prod_a * t
        acc = U * prod_a
        for b in range(D):
            term = e[b][int(c[i, b])]
            for d in range(D):
                if d != b:
                    term = term * a[d][int(c[i, d])]
            acc = acc + term
        out.append(phi_rho * acc)
    return np.stack(out)


# ---------------------------------------------------------------------------
# Oracle state machine
# ---------------------------------------------------------------------------

class Oracle:
    """One lattice Boltzmann run on the CPU.

    State: species populations fa (M,Q,N), momentum populations f (Q,N),
    energy populations g (Q,N) when the energy lattice is on, coverages
    theta (K,N).  Node index n = x + nx (y + ny z).
    """

    def __init__(self, w):
        self.w = w
        self.D = w.lattice
        self.c = lattice_velocities(self.D)
        self.Q = self.c.shape[0]
        self.wt = lattice_weights(self.c)
        self.opp = np.array([self.Q - 1 - i for i in range(self.Q)])
        self.M = w.M
        self.N = w.nx * w.ny * w.nz
        self.shape = (w.nz, w.ny, w.nx)
        self.m = np.asarray(w.molar_mass, dtype=np.float64)
        self.m_min = float(self.m.min())
        self.phi = np.asarray(w.phi, dtype=np.float64).copy()
        self.tort = np.asarray(w.tort, dtype=np.float64).copy()
        self.Dv = w.d_visc if w.d_visc else self.D
        # R16: lattice unit system
        self.theta_ref = w.theta_ref
        self.c2 = R_U * w.T_ref / (self.m_min * w.theta_ref)     # (m/s)^2
        self.dt = w.dx / math.sqrt(self.c2)                      # s
        self.rho_unit = w.P_ref / self.c2                        # kg/m^3
        self.knudsen = (w.pore_radius is not None and w.pore_radius > 0.0
                        and math.isfinite(w.pore_radius))
        self.mech = w.mech
        self.energy = bool(w.energy_on)
        if self.energy:
            self.cv_lat = np.asarray(w.cv, dtype=np.float64) / self.c2
            self.uf_lat = np.asarray(w.u_form, dtype=np.float64) / self.c2
        self.T_field = np.asarray(w.T0, dtype=np.float64).copy()
        # electrode coupling (Section 4.2, R30): Phi_electrode (V) and the electrolyte
        # resistivity Omega(x) (Ohm m); dphi is the potential difference the rates see
        self.electrode = getattr(w, "electrode", None)
        self.i_v = np.zeros(self.N)
        self.i_a = np.zeros(self.N)
        self.phi_el = np.zeros(self.N)
        self.dphi = np.zeros(self.N)
        self.n_lines = w.ny * w.nz                       # x lines: node n lies on line n // nx
        self.line = np.arange(self.N) // w.nx
        self.line_end = np.arange(self.n_lines) * w.nx + (w.nx - 1)
        if self.electrode is not None:
            self.set_electrode_potential(self.electrode["phi_ed"])
        self.step_count = 0
        self._init_state()

    # ----- small helpers ---------------------------------------------------
    def RaT(self, T):
        """Lattice R_a T = theta_ref (m_min / m_a) (T / T_ref); shape (M, N)."""
        return self.theta_ref * (self.m_min / self.m)[:, None] * (np.asarray(T) / self.w.T_ref)[None, :]

    def composition(self, rho_a):
        """Section 2.1: Y_a, 1/m = sum Y_a/m_a, X_a = m Y_a / m_a."""
        rho_s = rho_a.sum(axis=0)
        Y = rho_a / rho_s
        inv_m = (Y / self.m[:, None]).sum(axis=0)
        X = (Y / self.m[:, None]) / inv_m
        return Y, 1.0 / inv_m, X

    def to_grid(self, a):
        return a.reshape(a.shape[:-1] + self.shape)

    def from_grid(self, a):
        return a.reshape(a.shape[:-3] + (self.N,))

    def shift_periodic(self, a, cvec):
        """value at x - c (pull) with periodic wrap on every axis."""
        g = self.to_grid(a)
        for ax in range(self.D):
            if cvec[ax] != 0:
                g = np.roll(g, int(cvec[ax]), axis=-1 - ax)
        return self.from_grid(g)

    def xcoord(self):
        return np.tile(np.arange(self.w.nx), self.w.ny * self.w.nz)

    def neighbour_value(self, a, cvec):
        """A(x + c) with periodic wrap; mirror ghost A(x) beyond non-periodic x ends (R9)."""
        out = self.shift_periodic(a, -np.asarray(cvec))
        if self.w.bc_lo != BC_PERIODIC or self.w.bc_hi != BC_PERIODIC:
            x = self.xcoord()
            if cvec[0] == 1:
                mask = x == self.w.nx - 1
                out = np.where(mask, a, out)
            elif cvec[0] == -1:
                mask = x == 0
                out = np.where(mask, a, out)
        return out

    def gradient(self, a, comp):
        """R9: d_comp A = 3 sum_i w_i c_i,comp A(x + c_i)."""
        acc = np.zeros_like(a)
        for i in range(self.Q):
            ci = self.c[i, comp]
            if ci == 0:
                continue
            acc = acc + self.wt[i] * ci * self.neighbour_value(a, self.c[i])
        return 3.0 * acc

    # ----- equilibria ------------------------------------------------------
    def species_eq(self, phi_rho_a, v, RaT):
        return species_equilibrium(self.c, phi_rho_a, v, RaT)

    def g_equilibrium(self, phi_rho, U, RT, v):
        return energy_equilibrium(self.c, phi_rho, U, RT, v)

    # ----- initial state ---------------------------------------------------
    def _init_state(self):
        w = self.w
        T = self.T_field
        RaT = self.RaT(T)
        P_lat = np.asarray(w.P0, dtype=np.float64) / w.P_ref
        X0 = np.asarray(w.X0, dtype=np.float64)
        rho_a = X0 * P_lat[None, :] / RaT                      # P_a = X_a P = rho_a R_a T
        zero = [np.zeros(self.N)] * self.D
        self.fa = np.stack([self.species_eq(self.phi * rho_a[a], zero, RaT[a]) for a in range(self.M)])
        Y, mmix, X = self.composition(rho_a)
        RT = (Y * RaT).sum(axis=0)
        rho = rho_a.sum(axis=0)
        self.f = (self.phi * rho) * product_form(self.c, zero, [RT] * self.D)
        if self.energy:
            U = (Y * (self.uf_lat[:, None] + self.cv_lat[:, None] * T[None, :])).sum(axis=0)
            self.g = self.g_equilibrium(self.phi * rho, U, RT, zero)
        else:
            self.g = None
        if self.mech is not None:
            self.theta = np.repeat(np.asarray(self.mech.theta0, dtype=np.float64)[:, None], self.N, axis=1)
        else:
            self.theta = np.zeros((0, self.N))

    # ----- macroscopic fields (stages S1-S5) --------------------------------
    def macro(self):
        """Moments, composition, temperature, coefficients and the species
        velocity solve at the current time level."""
        w, c, D, M = self.w, self.c, self.D, self.M
        phi = self.phi
        out = {}
        rho_a = self.fa.sum(axis=1) / phi                                  # eq density1
        jt = np.stack([(self.fa * c[None, :, d, None]).sum(axis=1) for d in range(D)], axis=1)  # (M,D,N)
        rho = self.f.sum(axis=0) / phi                                     # eq fdensity
        j = np.stack([(self.f * c[:, d, None]).sum(axis=0) for d in range(D)])  # eq f1momMomentum
        u = j / rho
        v = u / phi
        Y, mmix, X = self.composition(rho_a)
        if self.energy:
            E = self.g.sum(axis=0) / (phi * rho)                           # eq g0momTotalEnergy
            v2 = (v * v).sum(axis=0)
            cvm = (Y * self.cv_lat[:, None]).sum(axis=0)
            u0m = (Y * self.uf_lat[:, None]).sum(axis=0)
            T = (E - 0.5 * v2 - u0m) / cvm                                 # eq temperature (R7, R15)
        else:
            T = self.T_field
        RaT = self.RaT(T)
        RT = (Y * RaT).sum(axis=0)                                         # R = R_U / m
        P = rho * RT                                                       # eq eosIdealGas (R24)
        Ps = (rho_a * RaT).sum(axis=0)                                     # Dalton: sum_a rho_a R_a T
        # coefficients (Section 2.3 with R1, R2, R14, R21)
        Tr = T / w.T_ref
        Dab = w.D_ref_lat[:, :, None] * (Tr ** 1.5)[None, None, :] / Ps[None, None, :]
        tau_ab = np.zeros((M, M, self.N), dtype=Dab.dtype)        # dtype follows the inputs (complex
        inv_tau_ab = np.zeros((M, M, self.N), dtype=Dab.dtype)    # for the complex-step tangent)
        for a in range(M):
            for b in range(M):
                if a != b:
                    tau_ab[a, b] = Dab[a, b] * (self.m[b] / mmix) / RaT[a]
                    inv_tau_ab[a, b] = 1.0 / tau_ab[a, b]
        inv_tau_a = np.stack([sum(Y[b] * inv_tau_ab[a, b] for b in range(M) if b != a) for a in range(M)])
        beta = inv_tau_a / (2.0 + inv_tau_a)                               # eq betaa: dt / (2 tau_a + dt)
        if self.knudsen:
            d0 = 2.0 * w.pore_radius
            Dk = (phi / self.tort)[None, :] * (d0 / (3.0 * w.dx)) * np.sqrt(8.0 * RaT / math.pi)
            inv_tau_k = RaT / Dk
        else:
            inv_tau_k = np.zeros((M, self.N))
        # R4: second-order species momenta, one M x M solve per direction and node
        A = np.zeros((self.N, M, M), dtype=np.result_type(inv_tau_a, inv_tau_k))
        for a in range(M):
            for b in range(M):
                if a == b:
                    A[:, a, a] = 1.0 + 0.5 * inv_tau_a[a] + 0.5 * inv_tau_k[a]
                else:
                    A[:, a, b] = -0.5 * Y[a] * inv_tau_ab[a, b]
        rhs = np.transpose(jt, (2, 0, 1))                                  # (N, M, D)
        jsol = np.linalg.solve(A, rhs)                                     # (N, M, D)
        ja = np.transpose(jsol, (1, 2, 0))                                 # (M, D, N)
        Fk = -(ja * inv_tau_k[:, None, :]).sum(axis=0)                     # eq netKnudsenForce
        with np.errstate(divide="ignore", invalid="ignore"):
            ua = np.where(rho_a[:, None, :] > 0.0, ja / rho_a[:, None, :], u[None, :, :])   # R19
        out.update(rho_a=rho_a, jt=jt, rho=rho, j=j, u=u, v=v, Y=Y, m=mmix, X=X, T=T, RaT=RaT,
                   RT=RT, P=P, Ps=Ps, tau_ab=tau_ab, inv_tau_ab=inv_tau_ab, inv_tau_a=inv_tau_a, beta=beta,
                   inv_tau_k=inv_tau_k, ja=ja, ua=ua, Va=ua - u[None], Fk=Fk)
        if self.energy:
            out["E"] = E
        return out

    # ----- S7: surface chemistry (Section 4, reading R13) -------------------
    def chemistry(self, mac):
        """Returns (src (M,N) = rho_dot_a^(f) delta_t in lattice phi*rho units, new theta)."""
        mech = self.mech
        M, K = self.M, mech.K
        S = M + K
        T = mac["T"]
        kf = mech.A_f[:, None] * np.exp(-mech.Ea_f[:, None] / (R_U * T[None, :]))      # (R, N)
        kb = mech.A_b[:, None] * np.exp(-mech.Ea_b[:, None] / (R_U * T[None, :]))
        zc = getattr(mech, "charge_z", None)
        if zc is not None:
            # R30: potential factors of the charge-transfer reactions
            zc = np.asarray(zc, dtype=np.float64)
            bct = np.asarray(mech.beta_ct, dtype=np.float64)
            fpot = F_C * self.dphi / (R_U * T)                                           # (N,)
            kf = kf * np.exp((bct * zc)[:, None] * fpot[None, :])
            kb = kb * np.exp(-((1.0 - bct) * zc)[:, None] * fpot[None, :])
        iv = np.zeros(self.N)
        nu_f = mech.nu_f.astype(np.float64)
        nu_b = mech.nu_b.astype(np.float64)
        stoich = (mech.nu_b - mech.nu_f).astype(np.float64)                            # (R, S)
        gam_k, a_k = self.surface_weights()                                              # (K,) per species
        ph = (np.zeros(K, dtype=int) if mech.surface_phase is None
              else np.asarray(mech.surface_phase, dtype=int))
        phi = self.phi
        h = self.dt / mech.n_sub
        c = (mac["rho_a"] * self.rho_unit / self.m[:, None]).T.copy()                    # (N, M) mol/m^3
        th = self.theta.T.copy()                                                         # (N, K)
        src = np.zeros((self.N, M))
        scale = np.concatenate([np.ones(M), gam_k])                                     # dC/dy

        def conc(cg, ts):
            return np.concatenate([cg, gam_k[None, :] * ts], axis=1)                     # (N, S)

        def rates(C):
            fwd = kf.T * np.prod(C[:, None, :] ** nu_f[None], axis=2)
            bwd = kb.T * np.prod(C[:, None, :] ** nu_b[None], axis=2)
            return fwd - bwd                                                             # (N, R)

        def drates(C):
            # d q_r / d C_s
            dq = np.zeros((self.N, mech.R, S))
            for s in range(S):
                nf = nu_f[:, s]
                nb = nu_b[:, s]
                Cf = C[:, None, :] ** nu_f[None]
                Cb = C[:, None, :] ** nu_b[None]
                Cf[:, :, s] = np.where(nf[None, :] > 0, nf[None, :] * C[:, None, s] ** np.maximum(nf - 1, 0)[None, :], 0.0)
                Cb[:, :, s] = np.where(nb[None, :] > 0, nb[None, :] * C[:, None, s] ** np.maximum(nb - 1, 0)[None, :], 0.0)
                dq[:, :, s] = kf.T * np.prod(Cf, axis=2) - kb.T * np.prod(Cb, axis=2)
            return dq

        wrow = np.concatenate([np.repeat(phi[:, None], M, axis=1),
                               np.repeat(gam_k[None, :], self.N, axis=0)], axis=1)       # (N, S)
        # volume factor of reaction r in the gas balances (eq totalFluidReactionRate):
        # a_s for a surface reaction (rate per unit surface), phi for a homogeneous
        # gas-phase reaction (rate per unit gas volume; eq dtrhoa balances phi rho_a)
        hom = (np.zeros(mech.R, dtype=bool) if mech.homogeneous is None
               else np.asarray(mech.homogeneous, dtype=bool))
        edge = (np.zeros(mech.R, dtype=bool) if mech.edge is None
                else np.asarray(mech.edge, dtype=bool))
        # phase of a surface reaction: the phase of its surface species (one phase each)
        sp_in = (mech.nu_f[:, M:] != 0) | (mech.nu_b[:, M:] != 0)                       # (R, K)
        r_phase = np.array([ph[sp_in[r]][0] if sp_in[r].any() else 0 for r in range(mech.R)])
        a_r = np.where(r_phase == 0, mech.a_s, mech.a_s2)
        vol = np.where(hom[None, :], phi[:, None], a_r[None, :])                        # (N, R)
        gas_st = stoich[:, :M]                                                           # (R, M)
        # eq totalSurfaceReactionRate: a coverage takes its surface's reactions per unit
        # area and the edge reactions scaled by l_TPB / a^(s) of its own surface
        surf_st = stoich[:, M:] * np.where(edge[:, None], mech.l_tpb / a_k[None, :], 1.0)   # (R, K)
        for _ in range(mech.n_sub):
            y0 = np.concatenate([c, th], axis=1)
            y = y0.copy()
            for _ in range(mech.n_newton):
                C = conc(y[:, :M], y[:, M:])
                q = rates(C)                                                             # (N, R)
                prod = np.concatenate([(vol * q) @ gas_st, q @ surf_st], axis=1)         # (N, S)
                F = wrow * (y - y0) - h * prod
                dq = drates(C) * scale[None, None, :]                                    # d q / d y
                J = np.zeros((self.N, S, S))
                idx = np.arange(S)
                J[:, idx, idx] = wrow
                J[:, :M, :] -= h * np.einsum("rs,nr,nrt->nst", gas_st, vol, dq)
                J[:, M:, :] -= h * np.einsum("rs,nrt->nst", surf_st, dq)
                y = y + np.linalg.solve(J, -F[:, :, None])[:, :, 0]
            C = conc(y[:, :M], y[:, M:])
            dxi = h * rates(C)                                                           # extents
            if zc is not None:
                iv += F_C * mech.l_tpb * (dxi @ zc) / self.dt                            # eq volumetricCurrent
            th = th + (dxi @ surf_st) / gam_k[None, :]
            dgas = (vol * dxi) @ gas_st                                                  # mol / m^3 total
            c = c + dgas / phi[:, None]
            src += dgas * self.m[None, :] / self.rho_unit
        if self.w.faradaic_rate is not None:
            fu, pr = self.w.faradaic_species
            r = np.asarray(self.w.faradaic_rate, dtype=np.float64) * self.dt             # mol/m^3 per step
            src[:, fu] -= r * self.m[fu] / self.rho_unit
            src[:, pr] += r * self.m[pr] / self.rho_unit
        self._iv = iv
        return src.T.copy(), th.T.copy()

    def electric_energy_source(self, iv):
        """U_source of R31 per node in lattice energy-density units."""
        mech = self.mech
        om = np.asarray(self.electrode["omega"], dtype=np.float64)
        om = np.tile(om, self.N // om.size) if om.size != self.N else om
        p_elec = np.abs(self.dphi) * iv                                                  # W/m^3
        p_om = (mech.a_s2 / mech.l_tpb) * iv * iv * om * self.w.dx                        # W/m^3
        return (p_om - p_elec) * self.dt / (self.rho_unit * self.c2)

    def set_electrode_potential(self, phi_ed):
        """Electrode potential of every x line (scalar or one per line), V."""
        self.ped = np.array(np.broadcast_to(np.asarray(phi_ed, dtype=np.float64), (self.n_lines,)))
        self.dphi = self.ped[self.line] - self.phi_el

    def match_current(self, mac):
        """R32: per-line secant on the electrode potential for the target end current."""
        el = self.electrode
        target = np.broadcast_to(np.asarray(el["target_ia"], dtype=np.float64), (self.n_lines,))

        def end_current(p_line):
            self.dphi = p_line[self.line] - self.phi_el
            self.chemistry(mac)                                  # trial: the state is not changed
            ia, _ = self.charge_transport(self._iv)
            return ia[self.line_end] - target

        p0 = self.ped.copy()
        f0 = end_current(p0)
        p1 = p0 + 0.01
        for _ in range(int(el["n_secant"])):
            f1 = end_current(p1)
            d = f1 - f0
            p2 = np.where(d != 0.0, p1 - f1 * (p1 - p0) / np.where(d != 0.0, d, 1.0), p1)
            p0, f0, p1 = p1, f1, p2
        self.set_electrode_potential(p1)

    def charge_transport(self, iv):
        """eqs areaCurrentDensity and electrolytePotential along x (R30): the area current
        density I^(a) and the electrolyte potential of every node from the volumetric
        current I^(v) (A/m^3), dx in metres, Omega(x) in Ohm m."""
        dx = self.w.dx
        om = np.asarray(self.electrode["omega"], dtype=np.float64)                      # (nx,)
        ia = np.cumsum(self.to_grid(iv) * dx, axis=-1)                                   # A/m^2
        pel = np.cumsum(ia * om * dx, axis=-1)                                           # V
        return self.from_grid(ia), self.from_grid(pel)

    def surface_energy(self, theta, T):
        """Internal energy of the adsorbed phase per unit volume, lattice units
        (eq temperatureCell, adsorbed part): a_s rho^(s) sum_k Y_k U_k(T) with
        rho^(s) Y_k = Gamma theta_k m_k and U_k = u_form_k + cv_k T.  Zero
        without adsorbed-phase thermo."""
        mech = self.mech
        if mech is None or mech.surf_cv is None:
            return np.zeros(self.N)
        m_k = np.asarray(mech.surf_mass, dtype=np.float64)
        Uk = (np.asarray(mech.surf_u_form, dtype=np.float64)[:, None]
              + np.asarray(mech.surf_cv, dtype=np.float64)[:, None] * np.asarray(T)[None, :])   # J/kg
        gam_k, a_k = self.surface_weights()
        dens = (a_k * gam_k * m_k)[:, None] * theta                                            # kg/m^3
        return (dens * Uk).sum(axis=0) / (self.rho_unit * self.c2)

    def surface_weights(self):
        """Site density Gamma and specific area a^(s) of each surface species' phase."""
        mech = self.mech
        ph = (np.zeros(mech.K, dtype=int) if mech.surface_phase is None
              else np.asarray(mech.surface_phase, dtype=int))
        gam_k = np.where(ph == 0, mech.gamma, mech.gamma2)
        a_k = np.where(ph == 0, mech.a_s, mech.a_s2)
        return gam_k, a_k

    # ----- one time step ---------------------------------------------------
    def step(self, n: int = 1):
        for _ in range(n):
            self._step()

    def _step(self):
        w, c, D, M, Q = self.w, self.c, self.D, self.M, self.Q
        phi = self.phi
        mac = self.macro()
        rho_a, rho, u, v = mac["rho_a"], mac["rho"], mac["u"], mac["v"]
        RaT, RT, Y = mac["RaT"], mac["RT"], mac["Y"]
        # S7 chemistry
        if self.electrode is not None and self.electrode.get("target_ia") is not None:
            self.match_current(mac)
        if self.mech is not None:
            src, theta_new = self.chemistry(mac)
        elif w.faradaic_rate is not None:
            src = np.zeros((M, self.N))
            fu, pr = w.faradaic_species
            r = np.asarray(w.faradaic_rate) * self.dt
            src[fu] -= r * self.m[fu] / self.rho_unit
            src[pr] += r * self.m[pr] / self.rho_unit
            theta_new = self.theta
        else:
            src = np.zeros((M, self.N))
            theta_new = self.theta
        # S8 species collision (eq finalNumericalEquationsReactive)
        feq = np.stack([self.species_eq(phi * rho_a[a], v, RaT[a]) for a in range(M)])
        fstar = np.zeros_like(feq)
        for a in range(M):
            pos = rho_a[a] > 0.0
            safe = np.where(pos, phi * rho_a[a], 1.0)
            xi = [np.where(pos, mac["ja"][a, d] / safe, 0.0) for d in range(D)]      # R3
            P = [xi[d] ** 2 + RaT[a] for d in range(D)]
            fstar[a] = np.where(pos[None, :], (phi * rho_a[a]) * product_form(c, xi, P), 0.0)
        zero = [np.zeros(self.N)] * D
        fk = np.stack([(phi * rho_a[a]) * product_form(c, zero, [RaT[a]] * D) for a in range(M)])
        new_fa = np.empty_like(self.fa)
        for a in range(M):
            Fa = np.zeros((Q, self.N))
            for b in range(M):
                if b != a:
                    Fa = Fa + mac["inv_tau_ab"][a, b] * (feq[b] - fstar[b])
            Fa = Y[a] * Fa + mac["inv_tau_k"][a] * (fstar[a] - fk[a])                 # eq fStar
            shape_src = product_form(c, v, [v[d] ** 2 + RaT[a] for d in range(D)])     # eq fsourceHetero
            beta = mac["beta"][a]
            new_fa[a] = (self.fa[a] + 2.0 * beta * (feq[a] - self.fa[a])
                         + (beta - 1.0) * Fa + src[a] * shape_src)
        # S6 gradients for the Galilean correction (R9, R10)
        Afield = [rho * u[d] * (1.0 - 3.0 * RT) - rho * u[d] ** 3 / phi ** 2 for d in range(D)]
        G = [self.gradient(Afield[d], d) for d in range(D)]
        # S9 momentum collision (eqs f_source, feqmix, Pex with R6, R11)
        nu = w.nu_lat
        omega = 1.0 / (nu / RT + 0.5)
        Pex = [RT + v[d] ** 2 + (2.0 - omega) / (2.0 * phi * rho * omega) * G[d] for d in range(D)]
        uex = [u[d] + mac["Fk"][d] / (omega * rho) for d in range(D)]
        fex = (phi * rho) * product_form(c, [uex[d] / phi for d in range(D)], Pex)
        ratio_m1 = src.sum(axis=0) / (phi * rho)                                       # rho_pc / rho - 1
        new_f = self.f + omega * (fex - self.f) + ratio_m1 * fex
        # S10 energy collision (eqs g, gstar, gstareq1mom, interdiffusion, corrFourier, qex)
        if self.energy:
            omega1 = 1.0 / (nu / (w.prandtl * RT) + 0.5)
            T = mac["T"]
            Ua = self.uf_lat[:, None] + self.cv_lat[:, None] * T[None, :]
            Umix = (Y * Ua).sum(axis=0)
            Ha = Ua + RaT
            geq = self.g_equilibrium(phi * rho, Umix, RT, v)
            q = np.stack([(self.g * c[:, d, None]).sum(axis=0) for d in range(D)])
            Pt = np.zeros((D, D, self.N))
            for a in range(D):
                for b in range(D):
                    Pt[a, b] = (self.f * (c[:, a] * c[:, b])[:, None]).sum(axis=0)
            P = mac["P"]
            Hmix = Umix + RT
            v2 = (v * v).sum(axis=0)
            dY = [[self.gradient(Y[a], d) for d in range(D)] for a in range(M)]
            Qv = []
            for al in range(D):
                qeq = rho * u[al] * (Hmix + 0.5 * v2)                                  # eq geq1mom
                corr = np.zeros(self.N)
                for be in range(D):
                    Peq = phi * rho * v[al] * v[be] + (phi * P if al == be else 0.0)    # eq Peq
                    corr = corr + v[be] * (Pt[al, be] - Peq)
                ubar = sum(Y[b] * mac["ua"][b, al] for b in range(M))
                diff = sum(Ha[a] * Y[a] * (mac["ua"][a, al] - ubar) for a in range(M))
                four = sum(Ha[a] * dY[a][al] for a in range(M))
                Qa = ((omega - omega1) * (q[al] - qeq - corr) + omega1 * rho * diff
                      + 0.5 * (2.0 - omega1) * P * phi * four
                      - 0.5 * (omega - omega1) * v[al] * G[al])
                Qv.append(Qa)
            new_g = self.g + omega * (geq - self.g)
            for i in range(Q):
                if int(np.abs(c[i]).sum()) == 1:
                    new_g[i] = new_g[i] + 0.5 * sum(c[i, d] * Qv[d] for d in range(D))
            if self.mech is not None or w.faradaic_rate is not None:
                # eqs temperatureCell, InternalEnergyCell_PC, g0mom_source, g_source (R27): the
                # unified internal energy (fluid + adsorbed phase, one T) is kept through the
                # chemistry, so the fluid's phi rho^pc U^pc = phi rho U + (E_s before - E_s after);
                # g^eq,source is g^eq with (rho^pc, U^pc), pre-collision v and RT.
                phirho_pc = phi * rho + src.sum(axis=0)
                dEs = self.surface_energy(self.theta, T) - self.surface_energy(theta_new, T)
                if (self.electrode is not None and self.mech is not None
                        and getattr(self.mech, "charge_z", None) is not None):
                    dEs = dEs + self.electric_energy_source(self._iv)                   # R31
                U_pc = (phi * rho * Umix + dEs) / phirho_pc
                new_g = new_g + (self.g_equilibrium(phirho_pc, U_pc, RT, v) - geq)
        else:
            new_g = None
        # S11 streaming + boundary conditions
        self.fa = np.stack([self.stream(new_fa[a], ("species", a), mac) for a in range(M)])
        self.f = self.stream(new_f, ("momentum",), mac)
        if self.energy:
            self.g = self.stream(new_g, ("energy",), mac)
        self.theta = theta_new
        if self.electrode is not None:
            self.i_v = self._iv if self.mech is not None else np.zeros(self.N)
            self.i_a, self.phi_el = self.charge_transport(self.i_v)
            self.dphi = self.ped[self.line] - self.phi_el
        self.step_count += 1

    # ----- S11 ---------------------------------------------------------------
    def inlet_eq(self, which, side, mac):
        """Equilibrium of the prescribed inlet state moving with the node velocity u(x, t) (R17)."""
        w = self.w
        X = np.asarray(w.inlet_lo_X if side == "lo" else w.inlet_hi_X, dtype=np.float64)
        Tin = np.full(self.N, w.inlet_T)
        RaT = self.RaT(Tin)
        Plat = w.inlet_P / w.P_ref
        rho_a = X[:, None] * Plat / RaT
        Y, mmix, _ = self.composition(rho_a)
        RT = (Y * RaT).sum(axis=0)
        rho = rho_a.sum(axis=0)
        v = mac["u"] / self.phi
        if which[0] == "species":
            a = which[1]
            return self.species_eq(self.phi * rho_a[a], v, RaT[a])
        if which[0] == "momentum":
            return (self.phi * rho) * product_form(self.c, [v[d] for d in range(self.D)],
                                                   [RT + v[d] ** 2 for d in range(self.D)])
        # energy lattice (R17, energy part): the inlet prescribes the temperature of what
        # enters; the entering energy populations are the equilibrium at the inlet
        # temperature of the mixture that is at the node (its density and composition at
        # step t), moving with the node velocity
        Yn = mac["Y"]
        RaTn = self.RaT(Tin)
        Un = (Yn * (self.uf_lat[:, None] + self.cv_lat[:, None] * Tin[None, :])).sum(axis=0)
        RTn = (Yn * RaTn).sum(axis=0)
        return self.g_equilibrium(self.phi * mac["rho"], Un, RTn, v)

    def stream(self, post, which, mac):
        w, c = self.w, self.c
        new = np.stack([self.shift_periodic(post[i], c[i]) for i in range(self.Q)])
        if w.bc_lo == BC_PERIODIC and w.bc_hi == BC_PERIODIC:
            return new
        x = self.xcoord()
        for side, xb, missing_sign in (("lo", 0, 1), ("hi", w.nx - 1, -1)):
            kind = w.bc_lo if side == "lo" else w.bc_hi
            if kind == BC_PERIODIC:
                continue
            mask = x == xb
            miss = [i for i in range(self.Q) if c[i, 0] == missing_sign]
            if kind == BC_BOUNCEBACK:
                for i in miss:
                    new[i, mask] = post[self.opp[i], mask]
            elif kind == BC_OUTFLOW:
                xs = xb + missing_sign        # upstream neighbour inside the domain
                src_mask = x == xs
                for i in miss:
                    new[i, mask] = new[i, src_mask]
            elif kind == BC_INLET:
                eq = self.inlet_eq(which, side, mac)
                for i in miss:
                    new[i, mask] = eq[i, mask]
        return new

    # ----- outputs -----------------------------------------------------------
    def outlet_flux(self, steps, species=0):
        """Objective of the adjoint: J = (1/T) sum over the T steps of
        sum_{x = nx-1} j_{s,x} / m_s, with j_s the solved second-order species
        momentum (eq transform1) at the time level each step starts from
        (0..T-1), lattice units over kg/mol.  Advances the oracle by T steps."""
        outlet = (np.arange(self.N) % self.w.nx) == self.w.nx - 1
        acc = 0.0
        for _ in range(steps):
            ja = self.macro()["ja"]                                                      # (M, D, N)
            acc = acc + np.sum(ja[species, 0, outlet]) / self.m[species]
            self.step(1)
        return acc / steps

    def moments(self):
        """Macroscopic fields at the current time level (the library's moment set)."""
        mac = self.macro()
        return {
            "rho_a": mac["rho_a"], "X": mac["X"], "u": mac["u"], "T": mac["T"], "P": mac["P"],
            "rho": mac["rho"], "j_a": mac["ja"], "theta": self.theta.copy(),
        }
