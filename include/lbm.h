/*
 * lbm.h -- C ABI of the MI355X (gfx950) mean-field lattice Boltzmann library for
 * reacting multicomponent gas mixtures in porous media (Sawant & Karlin, "Mean
 * field lattice Boltzmann model for reactive mixtures in porous media").
 *
 * One time step advances, on every node:
 *   - M species populations with Stefan-Maxwell cross relaxation and Knudsen
 *     (dusty-gas) relaxation: Section 2, eqs finalNumericalEquationsReactive,
 *     betaa, tauab, taua, fStar, tauak, transform1;
 *   - the mixture momentum populations with the porosity-dependent extended
 *     equilibrium and the Knudsen force: Section 3.2, eqs f, feqmix, Pex, Peq,
 *     netKnudsenForce, f_source;
 *   - optionally the mixture energy populations: Section 3.3, eqs g, geq_i,
 *     gstar, gstareq1mom, interdiffusion, corrFourier, qex;
 *   - optionally the local heterogeneous surface-reaction source that couples
 *     gas and adsorbed species: Section 4, eqs totalFluidReactionRate,
 *     molarToMassRates, surfaceMoleFractions, totalSurfaceReactionRate,
 *     rho_pc, fsourceHetero;
 *   - optionally charge transfer at the triple-phase boundary with the 1-D
 *     charge transport along x, the electrical energy source and current
 *     control by the electrode potential: Sections 4.1-4.2, eqs
 *     volumetricCurrent, areaCurrentDensity, electrolytePotential.
 *
 * Conventions
 *   - Every entry point returns an lbm_status; nothing throws or aborts across
 *     the ABI.  lbm_last_error() returns a text for the last failure on a ctx.
 *   - Input arrays are host pointers and are copied; the caller keeps them.
 *     Output buffers are owned by the caller (host or device, as flagged).
 *   - The context owns every device allocation it makes (hipMalloc at init and
 *     set-up calls only; lbm_step allocates nothing).
 *   - A context is not thread-safe.  Work is queued on the HIP stream given in
 *     the configuration (NULL = the null stream); lbm_moments synchronises it.
 *   - Node index n = x + nx * (y + ny * z).  Field arrays are [component][node].
 *   - Lattice units delta_x = delta_t = 1; physical inputs are SI.
 *   - Population layout in HBM: [lattice][direction][node] FP64 (or FP32 with
 *     precision = LBM_FP32), lattices 0..M-1 species, M momentum, M+1 energy;
 *     direction i = sum_a (c_ia + 1) 3^a.  All arithmetic is FP64.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument (sizes, ranges, positivity of the product form) */
  LBM_ENOMEM = -2,     /* device allocation failed */
  LBM_EHIP = -3,       /* a HIP runtime call failed */
  LBM_ESTATE = -4,     /* call-order violation (e.g. set-up after the first step) */
  LBM_EUNSTABLE = -5   /* health check found a non-finite value */
} lbm_status;

/* x-axis boundary kinds; y and z are periodic. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_BOUNCEBACK = 1, LBM_BC_INLET = 2, LBM_BC_OUTFLOW = 3 };
enum { LBM_FP64 = 0, LBM_FP32 = 1 };   /* population storage (lbm_config.precision) */

/* lbm_moments field mask; rows are written in this order, each [rows][N] FP64. */
enum {
  LBM_MOM_RHO_SPECIES = 1 << 0, /* M rows: rho_a = sum_i f_ai / phi (eq density1)          */
  LBM_MOM_VELOCITY    = 1 << 1, /* D rows: u = j / rho of the momentum lattice             */
  LBM_MOM_TEMPERATURE = 1 << 2, /* 1 row : T in kelvin                                     */
  LBM_MOM_PRESSURE    = 1 << 3, /* 1 row : P = rho R T in units of P_ref (eq eosIdealGas)  */
  LBM_MOM_SPECIES_FLUX= 1 << 4, /* M*D rows [a][d]: second-order species momentum j_a     */
  LBM_MOM_COVERAGE    = 1 << 5, /* K rows: surface coverages theta_s                      */
  LBM_MOM_DENSITY     = 1 << 6, /* 1 row : rho = sum_i f_i / phi (eq fdensity)            */
  LBM_MOM_MOLE_FRACTION=1 << 7  /* M rows: X_a                                             */
};

typedef struct {
  int32_t dim;             /* 1, 2 or 3: D1Q3, D2Q9, D3Q27 (Section 2.2 product form)     */
  int32_t nx, ny, nz;      /* grid; unused trailing extents must be 1                      */
  int32_t n_species;       /* M, 2..5                                                      */
  int32_t energy_on;       /* 1: energy lattice and temperature from eq temperature        */
  int32_t bc_lo_x, bc_hi_x;/* LBM_BC_* at x = 0 and x = nx-1 (periodic must be both)       */
  int32_t precision;       /* LBM_FP64 (0): populations stored in FP64; LBM_FP32 (1): stored
                              in FP32, every step's arithmetic still FP64 (half the bytes)  */
  double dx_m;             /* lattice spacing, m                                            */
  double T_ref_K;          /* reference (maximum) temperature of the unit system, K         */
  double P_ref_Pa;         /* pressure unit, Pa                                             */
  double theta_ref;        /* lattice R T of the lightest species at T_ref (1/3 typical)   */
  double nu_lat;           /* kinematic viscosity, lattice units (eq mu with mu = rho nu)  */
  double prandtl;          /* Prandtl number (eq lambda)                                    */
  const double *molar_mass;/* [M] kg/mol                                                     */
  const double *D_ref_lat; /* [M*M] binary diffusivities, lattice units at (T_ref, P_ref);
                              symmetric, diagonal ignored; D_ab scales as T^1.5 / P         */
  const double *cv;        /* [M] J/(kg K), energy_on only (U_a = u_form_a + cv_a T)        */
  const double *u_form;    /* [M] J/kg,     energy_on only                                  */
  const double *inlet_lo_X;/* [M] inlet mole fractions at x = 0, or NULL                    */
  const double *inlet_hi_X;/* [M] inlet mole fractions at x = nx-1, or NULL                 */
  double inlet_P_Pa;       /* inlet pressure, Pa                                            */
  double inlet_T_K;        /* inlet temperature, K                                          */
  void *hip_stream;        /* hipStream_t of the caller, or NULL                            */
} lbm_config;

/* Surface mechanism on one reactive surface (Section 4): K surface species
 * (index 0 of the surface block is the vacancy), R reversible mass-action
 * reactions q_r = kf prod C^nu_f - kb prod C^nu_b [mol m^-2 s^-1] with C the gas
 * concentration [mol m^-3] or Gamma theta [mol m^-2]; k = A exp(-Ea / (R_U T)).
 * The local update is backward Euler over n_sub sub-steps, each with n_newton
 * Newton iterations (dense LU with partial pivoting), followed by an
 * extent-based conservative update of gas and coverages. */
typedef struct {
  int32_t n_surface;       /* K (2..10)                                                    */
  int32_t n_reactions;     /* R (1..24)                                                    */
  int32_t n_sub, n_newton; /* fixed iteration counts (>= 1)                                */
  const int32_t *nu_f;     /* [R*(M+K)] reactant coefficients, 0..3                        */
  const int32_t *nu_b;     /* [R*(M+K)] product coefficients, 0..3                         */
  const double *A_f, *Ea_f;/* [R] SI (mol-based) pre-factor, J/mol                         */
  const double *A_b, *Ea_b;
  double gamma;            /* site density Gamma, mol/m^2 (eq surfaceMoleFractions)        */
  double a_s;              /* specific surface area a^(s), 1/m (eq totalFluidReactionRate) */
  const double *surf_mass; /* [K] kg/mol (mass bookkeeping; adsorbed-phase energy)         */
  const double *theta0;    /* [K] initial coverages, applied to every node                 */
  const double *surf_cv;   /* [K] J/(kg K) or NULL: adsorbed-phase internal energy         */
  const double *surf_u_form;/* [K] J/kg or NULL: U_k = u_form_k + cv_k T (eq temperatureCell).
                              With the energy lattice on, the chemistry keeps the unified
                              internal energy (fluid + adsorbed phase at one T, eq
                              InternalEnergyCell_PC) and the energy collision takes
                              g^eq,source - g^eq (eqs g0mom_source, g_source); surf_cv NULL
                              means no adsorbed-phase energy (surf_mass required otherwise) */
  const int32_t *homogeneous;/* [R] or NULL (all surface): 1 marks a homogeneous gas-phase
                              reaction (eqs sumRhoDot, totalFluidReactionRate): gas species
                              only, zero net mass; its mass-action rate is per unit gas
                              volume (mol m^-3 s^-1 with C the gas concentrations), so it
                              enters the gas balances with phi instead of a_s            */
  /* Second surface phase and triple-phase-boundary (TPB) edge (eqs totalSurfaceReactionRate,
   * totalSurfaceReactionRateTPB_electrode/_electrolyte).  surface_phase [K] (NULL: all 0)
   * assigns each surface species to phase 0 (gamma, a_s) or phase 1 (gamma2, a_s2); each
   * phase has its own vacancy and theta0 sums to 1 per phase.  A surface reaction's surface
   * species lie on one phase and balance its sites.  edge [R] (NULL: none) marks TPB
   * reactions among adsorbed species of both phases (no gas species, sites balanced per
   * phase) with a mass-action rate per unit edge length; l_tpb is the edge length per unit
   * volume (1/m^2), so a coverage of phase k takes l_tpb / a^(s)_k times the edge rate. */
  const int32_t *surface_phase;
  double gamma2;           /* site density of phase 1, mol/m^2                             */
  double a_s2;             /* specific surface area of phase 1, 1/m                        */
  const int32_t *edge;
  double l_tpb;            /* TPB length per unit volume, 1/m^2                            */
  /* Charge transfer at the TPB (Section 4.1, eq volumetricCurrent).  charge_z [R] (NULL: none)
   * is the number of electrons the forward direction of an edge reaction releases into the
   * electrode (-4..4; only edge reactions may carry charge); beta_ct [R] (required with
   * charge_z) the symmetry factor in [0, 1].  With dPhi = Phi_electrode - Phi_electrolyte at
   * the node, the mass-action constants become k_f exp(beta z F dPhi / (R_U T)) and
   * k_b exp(-(1 - beta) z F dPhi / (R_U T)) (dPhi = 0 without lbm_set_electrode), and the
   * step's volumetric current I^(v) = F l_TPB sum_r z_r xi_r / dt (A/m^3, extents xi_r per
   * unit TPB length over the step) is kept for lbm_get_charge.                            */
  const int32_t *charge_z;
  const double *beta_ct;
} lbm_mechanism;

/* Creates a context for a rectangular grid.  X0 [M][N] mole fractions, P0 [N]
 * pressure (Pa) or NULL for P_ref, T0 [N] temperature (K; the prescribed field
 * when energy_on == 0).  Populations are set to the equilibria of Section 2.2
 * and 3 at zero velocity with porosity 1 (lbm_set_porous_field rebuilds them).
 * Fails with LBM_EINVAL when the product form would not be positive
 * (R_a T > 1 for some species), when a mole fraction row does not sum to 1 or
 * when sizes are inconsistent. */
int lbm_init(const lbm_config *cfg, const double *X0, const double *P0, const double *T0,
             lbm_ctx **out);

/* Same as lbm_init for dim == 1 on n_cols independent packed columns of lengths
 * col_len[c] (N = sum col_len).  Every column gets the x boundary kinds of cfg at
 * its own ends (periodic is not allowed).  Used for batched 1-D button cells. */
int lbm_init_columns(const lbm_config *cfg, int32_t n_cols, const int32_t *col_len,
                     const double *X0, const double *P0, const double *T0, lbm_ctx **out);

/* Porosity phi [N] in (0,1], tortuosity tort [N] (NULL = 1) and the pore radius
 * r_p (m) of the Knudsen diffusivity D^k_a = (phi/tort)(2 r_p/3) sqrt(8 R_U T /(pi m_a))
 * (Section 5.1); r_p <= 0 or infinite switches Knudsen diffusion off.  Rebuilds
 * the initial populations; only valid before the first lbm_step (LBM_ESTATE). */
int lbm_set_porous_field(lbm_ctx *ctx, const double *phi, const double *tort, double pore_radius_m);

/* Installs the surface mechanism (NULL removes it) and sets the coverages to
 * theta0.  Only valid before the first lbm_step. */
int lbm_set_mechanism(lbm_ctx *ctx, const lbm_mechanism *mech);

/* Chemistry kernel used for an installed mechanism.  LBM_CHEM_SPECIALIZED
 * (default): the first step runs the generic kernel; before the second step
 * the library generates a kernel with the mechanism's stoichiometry and
 * Arrhenius constants written in and compiles it for gfx950 with hiprtc (once
 * per mechanism and process; a failed compilation makes that lbm_step return
 * LBM_EHIP).  It solves each Newton system with a sparse LU in an elimination
 * order chosen on Newton matrices sampled from the state after the first step,
 * and falls back, per node, to a dense LU with partial pivoting wherever
 * partial pivoting would exchange rows.  LBM_CHEM_GENERIC runs the precompiled
 * kernel that reads the mechanism from device tables (dense LU with partial
 * pivoting) on every step.  Both compute the backward-Euler update of
 * Section 4; they agree to rounding.  LBM_CHEM_SPECIALIZED_2W is the generated
 * kernel compiled for two waves per SIMD: its registers are capped at 256 and
 * what does not fit spills to scratch memory, which pays where the nodes fill
 * barely more than one wave per SIMD (the batched 1-D columns); same results
 * bitwise as LBM_CHEM_SPECIALIZED. */
enum { LBM_CHEM_SPECIALIZED = 0, LBM_CHEM_GENERIC = 1, LBM_CHEM_SPECIALIZED_2W = 2 };
int lbm_set_chem_kernel(lbm_ctx *ctx, int32_t kind);

/* Prescribed volumetric Faradaic source rate [N] (mol m^-3 s^-1) that consumes
 * species `fuel` and produces species `product` (explicit, added to the
 * chemistry source; NULL removes it).  Only valid before the first lbm_step. */
int lbm_set_faradaic_source(lbm_ctx *ctx, const double *rate, int32_t fuel, int32_t product);

/* Electrode coupling and 1-D charge transport along x (Section 4.2, eqs electrodePotential,
 * areaCurrentDensity, electrolytePotential).  The x lines are the ny nz rows of a regular
 * grid (line y + ny z) or the packed columns of lbm_init_columns (in column order).
 * phi_electrode: host [n_lines] potential of the electrode phase of each line, V (constant
 * along the line); omega: host [N] electrolyte resistivity at each node, Ohm m (>= 0); both
 * copied.  phi_electrode NULL switches the coupling off.  After each step's chemistry the
 * library integrates every line from its first node cell by cell (rectangle rule,
 * Phi_electrolyte = 0 before the first cell): I^(a)(x) = sum I^(v) dx and
 * Phi_electrolyte(x) = sum I^(a) Omega dx; the next step's charge-transfer rates see
 * dPhi = phi_electrode - Phi_electrolyte(x) (dPhi = phi_electrode before the first
 * integration).  May be called between steps (e.g. to sweep the potential: the
 * electrolyte potential is kept); it drops a captured step graph.  Snapshots (lbm_save)
 * carry the electrode state.                                                              */
int lbm_set_electrode(lbm_ctx *ctx, const double *phi_electrode, const double *omega);

/* Copies to host [N] arrays (each may be NULL) the last step's volumetric current I^(v)
 * (A/m^3), area current density I^(a) (A/m^2) and electrolyte potential (V); synchronizes
 * the stream.  Arrays the installed model does not produce are zero.  LBM_ESTATE without a
 * charge-transfer mechanism or an electrode.                                               */
int lbm_get_charge(lbm_ctx *ctx, double *iv, double *ia, double *phi_el);

/* Current control (Section 4.2: the electrode potential found by the secant method so that
 * the current matches a target).  target_ia: host [n_lines] area current density in A/m^2
 * wanted at the last node of each x line; NULL switches the control off.  Each step, after
 * the species kernel and before its chemistry, the library runs 1 + n_secant trial
 * chemistry passes (state unchanged, current only) with the line's charge integration:
 * iterates start at the line's present electrode potential and 10 mV above it, then
 * n_secant secant updates (none on a line whose two last currents are equal); the step
 * runs at the last iterate, which becomes the line's electrode potential
 * (lbm_get_electrode_potential).  n_secant in 1..64.  Needs lbm_set_electrode and a
 * charge-transfer mechanism (LBM_ESTATE otherwise); drops a captured step graph.        */
int lbm_set_current_target(lbm_ctx *ctx, const double *target_ia, int32_t n_secant);

/* Copies the electrode potential of each x line (host [n_lines], V); synchronizes the
 * stream.  LBM_ESTATE without an electrode.                                                */
int lbm_get_electrode_potential(lbm_ctx *ctx, double *phi_line);

/* Advances n_steps time steps, asynchronously on the configured stream.  One step is
 * the method's update of every lattice at every node (Sections 2.3, 3 and 4): stream
 * (pull) with the boundary conditions, moments and composition, temperature (eq
 * temperature), the species-momentum solve (eq transform1), the species collision (eq
 * finalNumericalEquationsReactive, with the reaction populations of eq fsourceHetero),
 * the local chemistry (Section 4) and the momentum and energy collisions (eqs f_source,
 * g_source).  n_steps >= 0; returns LBM_EHIP when a launch fails (the context is then
 * unusable).  Allocates nothing once the run-time generated kernels exist: the step
 * after the first compiles the mechanism's chemistry kernel, and the first fused
 * launch (lbm_set_persistent) compiles that kernel and sizes its buffers. */
int lbm_step(lbm_ctx *ctx, int64_t n_steps);

/* Graph step loop: with steps_per_graph = G (even, >= 2), lbm_step captures G
 * consecutive steps into a HIP graph once the run is past its first step (and,
 * with the generated chemistry kernel, once that kernel exists) and then
 * replays the graph for every whole G-step block; the remaining steps and any
 * step that would break the buffer parity run as plain launches.  Results are
 * bitwise those of plain launches.  Needs a non-null stream in the
 * configuration (LBM_EINVAL otherwise); 0 switches it off (default).  Per-kernel
 * timing (lbm_get_timing) covers the plain-launch steps only.  For launch-bound
 * runs such as the batched 1-D columns. */
int lbm_set_graph(lbm_ctx *ctx, int32_t steps_per_graph);

/* Persistent launch of one-dimensional lattices (packed columns of lbm_init_columns,
 * or a D1Q3 grid): with steps_per_launch = S (odd, 1..7) lbm_step advances the run S
 * whole steps per launch of one fused kernel, compiled at run time with the
 * context's constants and the mechanism's chemistry.  Each wave of 64 lanes owns
 * 64 - 4 S consecutive nodes and carries a window of 64 nodes (2 S more on either
 * side) through the S steps in registers: species lattices with their reaction
 * populations (Section 2.3, eqs finalNumericalEquationsReactive, fsourceHetero), the
 * node chemistry (Section 4) and the momentum lattice (eqs Pex, feqmix, f_source),
 * the same arithmetic in the same order as the separate kernels.  A step at a node
 * depends on the previous state within two nodes, so only the window's inner nodes
 * are stored; nothing is exchanged between waves within a launch.  waves_per_block
 * (1, 2 or 4) sets the workgroup size.  Covers isothermal D1Q3 runs with FP64
 * populations, closed x ends, no electrode coupling, and either no chemistry or a
 * mechanism with the generated chemistry kernel (with or without a Faradaic
 * source); LBM_EINVAL otherwise.  Steps before the chemistry kernel exists (the
 * first step) and a remainder shorter than S run the separate kernels; with the
 * graph step loop the graph holds whole launches (its length rounds up to a
 * multiple of 2 S).  0 switches it off (default). */
int lbm_set_persistent(lbm_ctx *ctx, int32_t steps_per_launch, int32_t waves_per_block);

/* Bound of the waits inside the D3Q27 species kernel, which runs two 64-node tiles
 * per workgroup and lets the waves of each tile meet at barriers of their own (a
 * counter in LDS that each wave polls).  A wave that has polled `polls` times
 * without the other waves of its tile arriving stops waiting and the step writes a
 * NaN population, so that lbm_get_diagnostics reports LBM_EUNSTABLE instead of the
 * kernel hanging.  Default 2^18 polls (milliseconds, against waits of microseconds).
 * Smaller values only serve tests of that failure path: 0 makes every such step
 * fail.  polls < 0: LBM_EINVAL.  Leaves the state alone; applies from the next step. */
int lbm_set_tile_wait_limit(lbm_ctx *ctx, int32_t polls);

/* One measured configuration of the step loop (lbm_autotune). */
typedef struct {
  int32_t fused;             /* 0: separate kernels, 1: fused persistent launch */
  int32_t chem_kernel;       /* chemistry kernel (LBM_CHEM_*) of the separate kernels */
  int32_t graph_steps;       /* graph step loop length (0: plain launches) */
  int32_t steps_per_launch;  /* fused: steps per launch */
  int32_t waves_per_block;   /* fused: waves per workgroup */
  double ms_per_step;        /* measured with HIP events on the context's stream */
} lbm_tune_entry;

/* Autotuner of the step loop: from the current state (past the first step;
 * LBM_ESTATE before), times about trial_steps steps (rounded up to whole launches)
 * of each configuration -- the separate kernels with plain launches and with the
 * graph step loop of 32 steps, with a mechanism also the graph loop with the
 * generated chemistry at two waves per SIMD (LBM_CHEM_SPECIALIZED_2W), and, where
 * lbm_set_persistent applies, the fused launch at 1, 3 and 5 steps per launch with
 * 1 or 2 waves per block -- restoring
 * the state before each, installs the fastest and restores the state again, so the
 * run continues from where it was.  Writes up to max_entries entries to table
 * (host memory, caller-owned) and their number to n_entries.  Needs a non-null
 * stream.  Synchronises the stream; allocates a host snapshot of the state
 * (lbm_save) for the call and compiles the fused variants it times. */
int lbm_autotune(lbm_ctx *ctx, int32_t trial_steps, lbm_tune_entry *table, int32_t max_entries,
                 int32_t *n_entries);

/* Gradient of an outlet-flux objective by the adjoint of the step (isothermal,
 * no surface mechanism or Faradaic source, D1Q3/D2Q9/D3Q27 grid with FP64
 * storage, not packed columns; LBM_EINVAL otherwise),
 * starting from the initial state (LBM_ESTATE after a step has been taken):
 *   J = (1/T) sum_{t=1..T} sum_{nodes with x = nx-1} j_{s,x}(t) / m_s,
 * with j_s the second-order species momentum of the species solve (eq
 * transform1) at the time level each of the T steps collides (0..T-1), in
 * lattice units divided by the molar mass in kg/mol.  Writes J, dJ/dphi per
 * node into grad_phi[N] (device pointer if out_on_device != 0, else host;
 * tortuosity held fixed, the initial populations and the inlet equilibria
 * included) and dJ/dr_p (1/m, 0 with Knudsen diffusion off).  Runs the T steps
 * forward in segments of K steps, checkpointing the start of every segment but the
 * last, whose states it keeps; the reverse sweep then takes the segments last
 * first, recomputing each earlier one from its checkpoint, so the forward work is
 * 2 T - K steps.  K is the largest the workspace budget allows (lbm_set_adjoint_memory;
 * K = T: every state kept, nothing recomputed).  The workspace, (K + 1) states and
 * the checkpoints and adjoint fields, is allocated for the call; LBM_ENOMEM when
 * even K = 1 does not fit.  Leaves the context at step T. */
int lbm_adjoint_outlet_flux(lbm_ctx *ctx, int64_t n_steps, int32_t species, double *J, double *grad_phi,
                            double *grad_rp, int32_t out_on_device);

/* Device-memory budget in bytes for the workspace of lbm_adjoint_outlet_flux; 0 (the
 * default) takes three quarters of the free device memory at the call.  Results do
 * not depend on it, only the recomputation does. */
int lbm_set_adjoint_memory(lbm_ctx *ctx, uint64_t bytes);

/* Writes the macroscopic fields selected by `mask` at the current time level,
 * SoA FP64 in mask-bit order, into out (device pointer if out_on_device != 0,
 * else host).  Synchronises the stream.  Returns LBM_EINVAL for an empty mask. */
int lbm_moments(lbm_ctx *ctx, uint32_t mask, double *out, int32_t out_on_device);

/* Number of rows lbm_moments writes for `mask` (so the caller can size out). */
int lbm_moment_rows(const lbm_ctx *ctx, uint32_t mask, int32_t *rows);

/* Conservation and health reduction (deterministic, fixed-order): per species
 * total sum_x sum_i f_ai, momentum-lattice mass and momentum, energy total,
 * minimum population and the count of non-finite populations. */
typedef struct {
  double species_mass[8];
  double mixture_mass;
  double mixture_momentum[3];
  double energy_total;
  double min_population;
  int64_t n_nonfinite;
  int64_t steps_done;
} lbm_diag;
int lbm_get_diagnostics(lbm_ctx *ctx, lbm_diag *out);

/* lbm_get_diagnostics for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * reduction and the same totals, bit for bit (the per-block partials are added in
 * block order on the device), with its scratch in a file-scope device array of
 * 2 MiB (2^18 doubles) instead of context memory, and no allocation of any kind.
 * Each GPU holds its own copy of that array until the process ends; it is set up
 * when the first context is created on the GPU (LBM_ESTATE before that).  A lattice
 * needs (ceil(N/256) + 1)(L + D + 2) doubles of it (L lattices, D dimensions: up to
 * about 6 million nodes for 6 lattices in 3-D, 9.5 million for 3 lattices in 2-D);
 * larger ones get LBM_EINVAL.
 * Every call on a GPU uses that GPU's one array, so calls that overlap on one GPU
 * (other host threads, other streams) race; nothing in it needs clearing between
 * calls.  Synchronises the context's stream. */
int lbm_get_diagnostics_static(lbm_ctx *ctx, lbm_diag *out);

/* Kernel time of the last lbm_step call's launches, measured with HIP events
 * on the configured stream: total ms of the call and, over its last <= 64
 * steps, the per-step averages of the species kernel, the chemistry kernel and
 * the mixture kernel (any output pointer may be NULL).  Enabled with
 * lbm_set_timing(ctx, 1). */
int lbm_set_timing(lbm_ctx *ctx, int32_t enable);
int lbm_get_timing(lbm_ctx *ctx, double *total_ms, double *species_ms, double *chem_ms,
                   double *mixture_ms);

/* Snapshot of the complete state (populations, node records, coverages, step
 * counter, and with an electrode installed its electrolyte potential, currents and
 * electrode potentials): call with buf == NULL to query *size.  Loading needs a context
 * set up the same way (lattice, mechanism, electrode coupling installed or not; the
 * resistivity, targets and other settings are configuration, not state). */
int lbm_save(lbm_ctx *ctx, void *buf, size_t *size);
int lbm_load(lbm_ctx *ctx, const void *buf, size_t size);

const char *lbm_last_error(const lbm_ctx *ctx);
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
