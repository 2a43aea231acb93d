"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice Boltzmann path runs in the HIP library
``_lib/liblbm.so``; importing this module fails loudly when it is missing.
The function names mirror the C entry points; ``Lattice`` is a thin owner of a
context.  Host arrays are numpy float64; outputs may also be torch CUDA
tensors (device pointers), and the HIP stream can be torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_EUNSTABLE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_BOUNCEBACK, BC_INLET, BC_OUTFLOW = 0, 1, 2, 3
CHEM_SPECIALIZED, CHEM_GENERIC, CHEM_SPECIALIZED_2W = 0, 1, 2
FP64, FP32 = 0, 1             # population storage; arithmetic is FP64 either way

MOM_RHO_SPECIES = 1 << 0
MOM_VELOCITY = 1 << 1
MOM_TEMPERATURE = 1 << 2
MOM_PRESSURE = 1 << 3
MOM_SPECIES_FLUX = 1 << 4
MOM_COVERAGE = 1 << 5
MOM_DENSITY = 1 << 6
MOM_MOLE_FRACTION = 1 << 7

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class lbm_config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_species", C.c_int32), ("energy_on", C.c_int32), ("bc_lo_x", C.c_int32),
        ("bc_hi_x", C.c_int32), ("precision", C.c_int32),
        ("dx_m", C.c_double), ("T_ref_K", C.c_double), ("P_ref_Pa", C.c_double),
        ("theta_ref", C.c_double), ("nu_lat", C.c_double), ("prandtl", C.c_double),
        ("molar_mass", _dp), ("D_ref_lat", _dp), ("cv", _dp), ("u_form", _dp),
        ("inlet_lo_X", _dp), ("inlet_hi_X", _dp), ("inlet_P_Pa", C.c_double),
        ("inlet_T_K", C.c_double), ("hip_stream", C.c_void_p),
    ]


class lbm_mechanism(C.Structure):
    _fields_ = [
        ("n_surface", C.c_int32), ("n_reactions", C.c_int32), ("n_sub", C.c_int32),
        ("n_newton", C.c_int32), ("nu_f", _ip), ("nu_b", _ip), ("A_f", _dp), ("Ea_f", _dp),
        ("A_b", _dp), ("Ea_b", _dp), ("gamma", C.c_double), ("a_s", C.c_double),
        ("surf_mass", _dp), ("theta0", _dp), ("surf_cv", _dp), ("surf_u_form", _dp),
        ("homogeneous", _ip), ("surface_phase", _ip), ("gamma2", C.c_double), ("a_s2", C.c_double),
        ("edge", _ip), ("l_tpb", C.c_double), ("charge_z", _ip), ("beta_ct", _dp),
    ]


class lbm_diag(C.Structure):
    _fields_ = [
        ("species_mass", C.c_double * 8), ("mixture_mass", C.c_double),
        ("mixture_momentum", C.c_double * 3), ("energy_total", C.c_double),
        ("min_population", C.c_double), ("n_nonfinite", C.c_int64), ("steps_done", C.c_int64),
    ]


class lbm_tune_entry(C.Structure):
    _fields_ = [("fused", C.c_int32), ("chem_kernel", C.c_int32), ("graph_steps", C.c_int32),
                ("steps_per_launch", C.c_int32), ("waves_per_block", C.c_int32), ("ms_per_step", C.c_double)]


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "lbm_init": ([C.POINTER(lbm_config), _dp, _dp, _dp, C.POINTER(vp)], C.c_int),
        "lbm_init_columns": ([C.POINTER(lbm_config), C.c_int32, _ip, _dp, _dp, _dp, C.POINTER(vp)], C.c_int),
        "lbm_set_porous_field": ([vp, _dp, _dp, C.c_double], C.c_int),
        "lbm_set_mechanism": ([vp, C.POINTER(lbm_mechanism)], C.c_int),
        "lbm_set_faradaic_source": ([vp, _dp, C.c_int32, C.c_int32], C.c_int),
        "lbm_set_chem_kernel": ([vp, C.c_int32], C.c_int),
        "lbm_set_electrode": ([vp, _dp, _dp], C.c_int),
        "lbm_get_charge": ([vp, _dp, _dp, _dp], C.c_int),
        "lbm_set_current_target": ([vp, _dp, C.c_int32], C.c_int),
        "lbm_get_electrode_potential": ([vp, _dp], C.c_int),
        "lbm_step": ([vp, C.c_int64], C.c_int),
        "lbm_set_graph": ([vp, C.c_int32], C.c_int),
        "lbm_set_persistent": ([vp, C.c_int32, C.c_int32], C.c_int),
        "lbm_set_tile_wait_limit": ([vp, C.c_int32], C.c_int),
        "lbm_autotune": ([vp, C.c_int32, C.POINTER(lbm_tune_entry), C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "lbm_adjoint_outlet_flux": ([vp, C.c_int64, C.c_int32, _dp, vp, _dp, C.c_int32], C.c_int),
        "lbm_set_adjoint_memory": ([vp, C.c_uint64], C.c_int),
        "lbm_moments": ([vp, C.c_uint32, vp, C.c_int32], C.c_int),
        "lbm_moment_rows": ([vp, C.c_uint32, _ip], C.c_int),
        "lbm_get_diagnostics": ([vp, C.POINTER(lbm_diag)], C.c_int),
        "lbm_get_diagnostics_static": ([vp, C.POINTER(lbm_diag)], C.c_int),
        "lbm_set_timing": ([vp, C.c_int32], C.c_int),
        "lbm_get_timing": ([vp, _dp, _dp, _dp, _dp], C.c_int),
        "lbm_save": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "lbm_load": ([vp, vp, C.c_size_t], C.c_int),
        "lbm_last_error": ([vp], C.c_char_p),
        "lbm_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()

EXPORTED = ["lbm_init", "lbm_init_columns", "lbm_set_porous_field", "lbm_set_mechanism",
            "lbm_set_chem_kernel", "lbm_set_faradaic_source", "lbm_set_electrode", "lbm_get_charge",
            "lbm_set_current_target", "lbm_get_electrode_potential", "lbm_step", "lbm_set_graph", "lbm_set_persistent", "lbm_set_tile_wait_limit", "lbm_autotune", "lbm_adjoint_outlet_flux", "lbm_set_adjoint_memory", "lbm_moments", "lbm_moment_rows",
            "lbm_get_diagnostics", "lbm_get_diagnostics_static", "lbm_set_timing", "lbm_get_timing", "lbm_save", "lbm_load",
            "lbm_last_error", "lbm_destroy"]


def _arr(a, dtype=np.float64):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, ctype=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


class Lattice:
    """Owner of one lbm_ctx.  Arguments follow the problem statement of the paper:
    molar masses, binary diffusivities, porosity/tortuosity, pore radius, T, P, X."""

    def __init__(self, dim, nx, ny, nz, molar_mass, D_ref_lat, X0, T0, P0=None, *, dx=1e-6,
                 T_ref=1073.0, P_ref=101325.0, theta_ref=1.0 / 3.0, nu_lat=0.05, prandtl=0.7,
                 energy_on=False, cv=None, u_form=None, bc_lo=BC_PERIODIC, bc_hi=BC_PERIODIC,
                 inlet_lo_X=None, inlet_hi_X=None, inlet_P=101325.0, inlet_T=1073.0,
                 stream=None, col_len=None, precision=FP64):
        self._keep = []
        m = _arr(molar_mass)
        M = int(m.shape[0])
        Dm = _arr(D_ref_lat).reshape(M, M)
        cfg = lbm_config()
        cfg.dim, cfg.nx, cfg.ny, cfg.nz = dim, nx, ny, nz
        cfg.n_species = M
        cfg.energy_on = 1 if energy_on else 0
        cfg.bc_lo_x, cfg.bc_hi_x = bc_lo, bc_hi
        cfg.precision = int(precision)
        cfg.dx_m, cfg.T_ref_K, cfg.P_ref_Pa, cfg.theta_ref = dx, T_ref, P_ref, theta_ref
        cfg.nu_lat, cfg.prandtl = nu_lat, prandtl
        arrays = dict(molar_mass=m, D_ref_lat=Dm, cv=_arr(cv), u_form=_arr(u_form),
                      inlet_lo_X=_arr(inlet_lo_X), inlet_hi_X=_arr(inlet_hi_X))
        for k, v in arrays.items():
            self._keep.append(v)
            setattr(cfg, k, _ptr(v))
        cfg.inlet_P_Pa, cfg.inlet_T_K = inlet_P, inlet_T
        cfg.hip_stream = stream
        self.cfg = cfg
        X0 = _arr(X0)
        T0 = _arr(T0)
        P0 = _arr(P0)
        ctx = C.c_void_p()
        if col_len is None:
            rc = _lib.lbm_init(C.byref(cfg), _ptr(X0), _ptr(P0), _ptr(T0), C.byref(ctx))
        else:
            cl = _arr(col_len, np.int32)
            rc = _lib.lbm_init_columns(C.byref(cfg), int(cl.shape[0]), _ptr(cl, C.c_int32), _ptr(X0),
                                       _ptr(P0), _ptr(T0), C.byref(ctx))
        self.ctx = ctx
        self.M, self.dim = M, dim
        self.n_lines = ny * nz if col_len is None else int(len(col_len))
        self.nx = nx
        self.N = int(X0.shape[-1])
        self.K = 0
        self._check(rc)

    # -- error handling --------------------------------------------------------
    def _check(self, rc):
        if rc != LBM_OK:
            msg = _lib.lbm_last_error(self.ctx).decode() if self.ctx else ""
            raise LBMError(rc, msg)

    def close(self):
        if getattr(self, "ctx", None):
            _lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ----------------------------------------------------------------
    def set_porous_field(self, phi, tort=None, pore_radius=float("inf")):
        phi = _arr(phi)
        tort = _arr(tort)
        self._check(_lib.lbm_set_porous_field(self.ctx, _ptr(phi), _ptr(tort), float(pore_radius)))

    def set_mechanism(self, mech):
        """mech: object with K, nu_f, nu_b, A_f, Ea_f, A_b, Ea_b, gamma, a_s, surf_mass, theta0,
        n_sub, n_newton and optionally surf_cv, surf_u_form, homogeneous, surface_phase,
        gamma2, a_s2, edge, l_tpb, charge_z, beta_ct (None removes the mechanism)."""
        if mech is None:
            self._check(_lib.lbm_set_mechanism(self.ctx, None))
            self.K = 0
            return
        keep = dict(nu_f=_arr(mech.nu_f, np.int32).ravel(), nu_b=_arr(mech.nu_b, np.int32).ravel(),
                    A_f=_arr(mech.A_f), Ea_f=_arr(mech.Ea_f), A_b=_arr(mech.A_b), Ea_b=_arr(mech.Ea_b),
                    surf_mass=_arr(mech.surf_mass), theta0=_arr(mech.theta0),
                    surf_cv=_arr(getattr(mech, "surf_cv", None)),
                    surf_u_form=_arr(getattr(mech, "surf_u_form", None)),
                    homogeneous=_arr(getattr(mech, "homogeneous", None), np.int32),
                    surface_phase=_arr(getattr(mech, "surface_phase", None), np.int32),
                    edge=_arr(getattr(mech, "edge", None), np.int32),
                    charge_z=_arr(getattr(mech, "charge_z", None), np.int32),
                    beta_ct=_arr(getattr(mech, "beta_ct", None)))
        st = lbm_mechanism()
        st.n_surface = int(mech.K)
        st.n_reactions = int(np.asarray(mech.nu_f).shape[0])
        st.n_sub, st.n_newton = int(mech.n_sub), int(mech.n_newton)
        st.nu_f = _ptr(keep["nu_f"], C.c_int32)
        st.nu_b = _ptr(keep["nu_b"], C.c_int32)
        st.homogeneous = _ptr(keep["homogeneous"], C.c_int32)
        st.surface_phase = _ptr(keep["surface_phase"], C.c_int32)
        st.edge = _ptr(keep["edge"], C.c_int32)
        st.charge_z = _ptr(keep["charge_z"], C.c_int32)
        st.beta_ct = _ptr(keep["beta_ct"])
        st.gamma2 = float(getattr(mech, "gamma2", 0.0) or 0.0)
        st.a_s2 = float(getattr(mech, "a_s2", 0.0) or 0.0)
        st.l_tpb = float(getattr(mech, "l_tpb", 0.0) or 0.0)
        for k in ("A_f", "Ea_f", "A_b", "Ea_b", "surf_mass", "theta0", "surf_cv", "surf_u_form"):
            setattr(st, k, _ptr(keep[k]))
        st.gamma, st.a_s = float(mech.gamma), float(mech.a_s)
        self._check(_lib.lbm_set_mechanism(self.ctx, C.byref(st)))
        self.K = int(mech.K)

    def set_chem_kernel(self, kind):
        """CHEM_SPECIALIZED (default), CHEM_GENERIC or CHEM_SPECIALIZED_2W (two waves per SIMD)."""
        self._check(_lib.lbm_set_chem_kernel(self.ctx, int(kind)))

    def set_faradaic_source(self, rate, fuel=0, product=1):
        rate = _arr(rate)
        self._check(_lib.lbm_set_faradaic_source(self.ctx, _ptr(rate), int(fuel), int(product)))

    def set_electrode(self, phi_electrode, omega):
        """Electrode potential (V; scalar or one per x line) and electrolyte resistivity
        (Ohm m; [N] per node, or [nx] repeated on every row of a regular grid) of the 1-D
        charge transport along x; phi_electrode None switches it off."""
        if phi_electrode is None:
            self._check(_lib.lbm_set_electrode(self.ctx, None, None))
            return
        ped = np.ascontiguousarray(np.broadcast_to(np.asarray(phi_electrode, dtype=np.float64),
                                                   (self.n_lines,)))
        om = _arr(omega).reshape(-1)
        if om.size != self.N:
            om = np.ascontiguousarray(np.tile(om, self.n_lines))
        if om.size != self.N:
            raise ValueError("omega must have N or nx entries")
        self._check(_lib.lbm_set_electrode(self.ctx, _ptr(ped), _ptr(om)))

    def set_current_target(self, target_ia, n_secant=6):
        """Area current density (A/m^2; scalar or one per x line) each step's electrode
        potentials are solved for; None switches the control off."""
        if target_ia is None:
            self._check(_lib.lbm_set_current_target(self.ctx, None, 0))
            return
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(target_ia, dtype=np.float64), (self.n_lines,)))
        self._check(_lib.lbm_set_current_target(self.ctx, _ptr(t), int(n_secant)))

    def electrode_potential(self):
        """Electrode potential of each x line, V."""
        out = np.empty(self.n_lines)
        self._check(_lib.lbm_get_electrode_potential(self.ctx, _ptr(out)))
        return out

    def charge(self):
        """(I^(v) A/m^3, I^(a) A/m^2, Phi_electrolyte V) of the last step, host float64 [N] each."""
        out = [np.empty(self.N) for _ in range(3)]
        self._check(_lib.lbm_get_charge(self.ctx, *(_ptr(o) for o in out)))
        return tuple(out)

    # -- run -------------------------------------------------------------------
    def step(self, n=1):
        self._check(_lib.lbm_step(self.ctx, int(n)))

    def adjoint_outlet_flux(self, n_steps, species=0, grad_out=None):
        """Runs n_steps from the initial state and returns (J, dJ/dphi [N], dJ/dr_p) for the
        outlet flux of `species` (see lbm_adjoint_outlet_flux).  grad_out: optional torch
        CUDA tensor of N float64 that receives dJ/dphi on the device."""
        J = C.c_double()
        grp = C.c_double()
        if grad_out is not None:
            self._check(_lib.lbm_adjoint_outlet_flux(self.ctx, int(n_steps), int(species), C.byref(J),
                                                     C.c_void_p(grad_out.data_ptr()), C.byref(grp), 1))
            return J.value, grad_out, grp.value
        g = np.zeros(self.N)
        self._check(_lib.lbm_adjoint_outlet_flux(self.ctx, int(n_steps), int(species), C.byref(J),
                                                 g.ctypes.data_as(C.c_void_p), C.byref(grp), 0))
        return J.value, g, grp.value

    def set_adjoint_memory(self, nbytes):
        """Workspace budget of adjoint_outlet_flux in bytes (0: 3/4 of the free device memory)."""
        self._check(_lib.lbm_set_adjoint_memory(self.ctx, int(nbytes)))

    def set_graph(self, steps_per_graph):
        """Replay whole blocks of `steps_per_graph` (even) steps as a HIP graph; 0 = off."""
        self._check(_lib.lbm_set_graph(self.ctx, int(steps_per_graph)))

    def set_persistent(self, steps_per_launch, waves_per_block=1):
        """Fused launch of `steps_per_launch` (odd) whole steps for 1-D lattices; 0 = off."""
        self._check(_lib.lbm_set_persistent(self.ctx, int(steps_per_launch), int(waves_per_block)))

    def set_tile_wait_limit(self, polls):
        """Bound (polls) of the species kernel's per-tile barrier waits; 0 fails every D3Q27 step."""
        self._check(_lib.lbm_set_tile_wait_limit(self.ctx, int(polls)))

    def autotune(self, trial_steps=200):
        """Times the step-loop configurations from the current state, installs the fastest
        and returns the table [(fused, graph_steps, steps_per_launch, waves_per_block,
        ms_per_step, chem_kernel)] (the state is left where it was)."""
        tab = (lbm_tune_entry * 16)()
        n = C.c_int32()
        self._check(_lib.lbm_autotune(self.ctx, int(trial_steps), tab, 16, C.byref(n)))
        return [(t.fused, t.graph_steps, t.steps_per_launch, t.waves_per_block, t.ms_per_step, t.chem_kernel)
                for t in tab[:n.value]]

    def moment_rows(self, mask):
        r = C.c_int32()
        self._check(_lib.lbm_moment_rows(self.ctx, mask, C.byref(r)))
        return r.value

    def moments(self, mask, out=None):
        """Host numpy [rows, N] by default; a torch CUDA tensor `out` receives them on device."""
        rows = self.moment_rows(mask)
        if out is None:
            out = np.empty((rows, self.N))
            self._check(_lib.lbm_moments(self.ctx, mask, out.ctypes.data_as(C.c_void_p), 0))
            return out
        self._check(_lib.lbm_moments(self.ctx, mask, C.c_void_p(out.data_ptr()), 1))
        return out

    def fields(self):
        """Dictionary of the standard macroscopic fields (host)."""
        M, D = self.M, self.dim
        mask = (MOM_RHO_SPECIES | MOM_VELOCITY | MOM_TEMPERATURE | MOM_PRESSURE | MOM_SPECIES_FLUX
                | MOM_DENSITY | MOM_MOLE_FRACTION | (MOM_COVERAGE if self.K else 0))
        a = self.moments(mask)
        o = 0
        out = {}
        for key, n in (("rho_a", M), ("u", D), ("T", 1), ("P", 1), ("j_a", M * D),
                       ("theta", self.K), ("rho", 1), ("X", M)):
            out[key] = a[o:o + n]
            o += n
        out["T"] = out["T"][0]
        out["P"] = out["P"][0]
        out["rho"] = out["rho"][0]
        out["j_a"] = out["j_a"].reshape(M, D, -1)
        return out

    def diagnostics(self, check=True):
        d = lbm_diag()
        rc = _lib.lbm_get_diagnostics(self.ctx, C.byref(d))
        if check:
            self._check(rc)
        return {"species_mass": np.array(d.species_mass[:self.M]), "mixture_mass": d.mixture_mass,
                "mixture_momentum": np.array(d.mixture_momentum[:self.dim]),
                "energy_total": d.energy_total, "min_population": d.min_population,
                "n_nonfinite": d.n_nonfinite, "steps_done": d.steps_done, "rc": rc}

    def diagnostics_static(self, check=True):
        """lbm_get_diagnostics_static: the same totals from the library's file-scope
        scratch, without any allocation (see include/lbm.h)."""
        d = lbm_diag()
        rc = _lib.lbm_get_diagnostics_static(self.ctx, C.byref(d))
        if check:
            self._check(rc)
        return {"species_mass": np.array(d.species_mass[:self.M]), "mixture_mass": d.mixture_mass,
                "mixture_momentum": np.array(d.mixture_momentum[:self.dim]),
                "energy_total": d.energy_total, "min_population": d.min_population,
                "n_nonfinite": d.n_nonfinite, "steps_done": d.steps_done, "rc": rc}

    def set_timing(self, on=True):
        self._check(_lib.lbm_set_timing(self.ctx, 1 if on else 0))

    def timing(self):
        t = [C.c_double() for _ in range(4)]
        self._check(_lib.lbm_get_timing(self.ctx, *[C.byref(x) for x in t]))
        return {"total_ms": t[0].value, "species_ms": t[1].value, "chem_ms": t[2].value,
                "mixture_ms": t[3].value}

    def save(self) -> bytes:
        size = C.c_size_t()
        self._check(_lib.lbm_save(self.ctx, None, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._check(_lib.lbm_save(self.ctx, buf, C.byref(size)))
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(_lib.lbm_load(self.ctx, buf, len(blob)))


def lattice_from_workload(w, stream=None, col_len=None, precision=FP64) -> Lattice:
    """Builds a Lattice from a workload description (attribute names as in workloads.synth)."""
    lat = Lattice(w.lattice, w.nx, w.ny, w.nz, w.molar_mass, w.D_ref_lat, w.X0, w.T0, w.P0,
                  dx=w.dx, T_ref=w.T_ref, P_ref=w.P_ref, theta_ref=w.theta_ref, nu_lat=w.nu_lat,
                  prandtl=w.prandtl, energy_on=w.energy_on, cv=w.cv, u_form=w.u_form,
                  bc_lo=w.bc_lo, bc_hi=w.bc_hi, inlet_lo_X=w.inlet_lo_X, inlet_hi_X=w.inlet_hi_X,
                  inlet_P=w.inlet_P, inlet_T=w.inlet_T, stream=stream, col_len=col_len, precision=precision)
    lat.set_porous_field(w.phi, w.tort, w.pore_radius if w.pore_radius is not None else float("inf"))
    if w.faradaic_rate is not None:
        lat.set_faradaic_source(w.faradaic_rate, *w.faradaic_species)
    if w.mech is not None:
        lat.set_mechanism(w.mech)
    el = getattr(w, "electrode", None)
    if el is not None:
        lat.set_electrode(el["phi_ed"], el["omega"])
        if el.get("target_ia") is not None:
            lat.set_current_target(el["target_ia"], el.get("n_secant", 6))
    return lat


def outlet_flux(phi, pore_radius, workload, n_steps, species=0, stream=None):
    """Outlet-flux objective J(phi, r_p) of `workload` (porosity and pore radius replaced)
    as a differentiable torch scalar: the forward runs the library, the backward returns
    the adjoint gradients (lbm_adjoint_outlet_flux).  phi: float64 tensor [N] (any device),
    pore_radius: float64 scalar tensor (metres)."""
    import torch

    class _OutletFlux(torch.autograd.Function):
        @staticmethod
        def forward(ctx, phi_t, rp_t):
            from dataclasses import replace
            w = replace(workload, phi=phi_t.detach().double().cpu().numpy(),
                        pore_radius=float(rp_t.detach().cpu()))
            lat = lattice_from_workload(w, stream=stream)
            dev = phi_t.device if phi_t.is_cuda else torch.device("cuda")
            g = torch.empty(lat.N, dtype=torch.float64, device=dev)
            J, g, grp = lat.adjoint_outlet_flux(n_steps, species, grad_out=g)
            lat.close()
            ctx.save_for_backward(g.to(phi_t.device), torch.tensor(grp, dtype=torch.float64, device=rp_t.device))
            return torch.tensor(J, dtype=torch.float64, device=phi_t.device)

        @staticmethod
        def backward(ctx, gJ):
            g, grp = ctx.saved_tensors
            return gJ * g, gJ * grp

    return _OutletFlux.apply(phi, pore_radius)
