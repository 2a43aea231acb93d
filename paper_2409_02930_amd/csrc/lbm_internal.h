// Internal declarations shared by the kernels and the host side of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#define LBM_MMAX 5          // gas species
#define LBM_KMAX 10         // surface species (vacancy included)
#define LBM_RMAX 24         // surface reactions
#define LBM_SMAX (LBM_MMAX + LBM_KMAX)

enum { BC_PERIODIC = 0, BC_BOUNCEBACK = 1, BC_INLET = 2, BC_OUTFLOW = 3 };

constexpr int kRec = 11;    // planes of the node records (velocity, species source, energy inlet)
constexpr int kRecSrc = 3;  // first plane of the species source
constexpr int kRecEin = 8;  // inlet nodes with the energy lattice: rho, U and R T of the node's
                            //   mixture at the inlet temperature (planes 8, 9, 10)

// Equilibrium state of a prescribed inlet mixture (lattice units).
struct InletState {
  double rho_a[LBM_MMAX];   // species densities X_a P / (R_a T)
  double RaT[LBM_MMAX];     // R_a T
  double rho;               // sum of rho_a
  double RT;                // mixture R T
  double U;                 // mixture internal energy (energy lattice)
  double T_K;               // inlet temperature, kelvin
};

// Everything the per-node stream/collide kernels read.  Passed by value.
struct KParams {
  int N, nx, ny, nz;
  int M, energy, bc_lo, bc_hi;
  int first_step;           // populations are stored post-stream: identity pull
  int knudsen;              // Knudsen relaxation on
  int chem;                 // a chemistry source is computed this step
  int need_v;               // node velocities are needed by the next step
  int src_prev;             // species pulls add the reaction populations of the previous step
  int fp32;                 // populations stored as float (arithmetic stays double)
  int tile_polls;           // bound of a tile barrier's wait in the species kernel (polls)
  int xcd_slabs;            // species kernel: XCD k takes the y slab k of every z plane (ny % 8 == 0,
                            //   nx a multiple of the block's nodes); 0: XCD k takes the k-th eighth
  int pad2;
  const int8_t *colflag;    // packed 1-D columns: bit0 = left end, bit1 = right end; NULL = grid
  double theta_ref, inv_T_ref, nu, prandtl;
  double mmin_over_m[LBM_MMAX];   // m_min / m_a
  double inv_m[LBM_MMAX];         // 1 / m_a
  double Dref[LBM_MMAX * LBM_MMAX];
  double imD[LBM_MMAX * LBM_MMAX];  // inv_m[b] / Dref[a][b]
  double cv[LBM_MMAX], uf[LBM_MMAX];   // lattice units (per kelvin, absolute)
  InletState inlet[2];            // x = 0 and x = nx - 1
  // populations [lattice][direction][node], double or float (fp32)
  const void *pin;
  void *pout;
  // static per-node fields
  const double *phi;        // porosity
  const double *kfac;       // (phi/tort) (d0 / 3 dx) sqrt(8/pi); D^k_a = kfac sqrt(R_a T)
  const double *Tfield;     // prescribed temperature (isothermal)
  // records written by the species kernel for the mixture / chemistry kernels
  double *rA;               // [D][N] rho u (1 - 3RT) - rho u^3 / phi^2
  double *rRT;              // [N] mixture R T
  double *rFk;              // [D][N] Knudsen force
  double *rrho;             // [M][N] species densities (chemistry input)
  double *rY;               // [M+2][N] mass fractions (energy lattice), then sum_a uf_a Y_a and
                            //   sum_a (cv_a + R_a / T) Y_a, so sum_a H_a(T) Y_a = row M + T row M+1
  double *rqd;              // [D][N] sum_a H_a Y_a (u_a - u_bar) (energy lattice)
  // ping-pong node records between consecutive steps, kRec planes of N doubles:
  //   planes 0..2 v = u/phi, planes 3..7 species source rho_dot_a dt (lattice units),
  //   planes 8..10 the energy-inlet state of inlet nodes (energy lattice only)
  const double *rec_prev;   // written by the previous step
  double *rec_cur;          // written by this step
  const double *T_prev;     // [N] temperature of the previous step (energy) or Tfield
  double *T_cur;            // energy only
  const double *srcsum_cur; // [N] sum_a source of this step (mixture mass source)
  // adsorbed-phase internal energy (energy lattice with a mechanism that has
  // surface thermo): E_s = sum_k theta_k (es_u[k] + es_c[k] T), lattice units
  int K, esrc;
  const double *theta;      // [K][N] coverages (after this step's chemistry in k_mixture)
  double *rEs;              // [N] E_s before this step's chemistry
  const double *uel;        // [N] electrical energy source of this step's chemistry, or NULL
  double es_u[LBM_KMAX], es_c[LBM_KMAX];
};

// Mechanism tables, kept in device memory (indexed by the run-time reaction).
struct ChemTables {
  double A_f[LBM_RMAX], Ea_f[LBM_RMAX], A_b[LBM_RMAX], Ea_b[LBM_RMAX];
  alignas(16) int8_t nu_f[LBM_RMAX][16];
  alignas(16) int8_t nu_b[LBM_RMAX][16];
  // gas-row weight of reaction r: w_r (a^(s) of its surface phase) or phi for a homogeneous one;
  // coverage-row weight of surface species k: 1, or l_TPB / a_k for an edge reaction
  double w_r[LBM_RMAX];
  double gam_k[LBM_KMAX], a_k[LBM_KMAX];   // site density and area of species k's phase
  double l_tpb;
  double beta_ct[LBM_RMAX];      // symmetry factor of a charge-transfer reaction
  int8_t kind[LBM_RMAX];         // 0 surface, 1 homogeneous gas-phase, 2 TPB edge
  int8_t charge_z[LBM_RMAX];     // electrons the forward direction releases into the electrode
};

struct ChemParams {
  int N, M, K, R;
  int n_sub, n_newton;
  int fuel, product;
  const ChemTables *tab;    // device
  double m[LBM_MMAX];       // kg/mol
  double gamma, a_s, rho_unit, dt, R_U;
  const double *rrho;       // [M][N]
  const double *T;          // [N]
  const double *phi;        // [N]
  const double *faradaic;   // [N] mol m^-3 s^-1 or NULL
  double *theta;            // [K][N] in place
  double *rec;              // node records of this step: source written to plane kRecSrc + a
  double *srcsum;           // [N]
  // charge transfer: dPhi = ped[n] - pel[n] (electrode minus electrolyte potential; pel
  // NULL: dPhi = 0); iv [N] receives the volumetric current (NULL: the mechanism has no
  // charge-transfer reaction)
  const double *ped, *pel;
  double F_C;
  double *iv;
  // electrical energy source (energy lattice on): uel[n] = (P_Omega - P_elec) dt in lattice
  // energy units, P_elec = |dPhi| I^(v), P_Omega = (a_el / l_TPB) I^(v)^2 omega[n] dx
  const double *omega;
  double a_el, dx, inv_e_unit;
  double *uel;
  int dry;                  // trial of the current control: write iv only
};

// Current control: per-line secant state (lines of ChargeParams).
struct SecantParams {
  int lines, stage, final_iter;
  const int *off;           // [lines + 1]
  const double *ia;         // [N] I^(a) of the trial
  const double *target;     // [lines] A/m^2
  double *p0, *f0, *p1;     // [lines] iterates and the current error of p0
  double *phi_line;         // [lines] electrode potential of the line
  double *ped_try, *ped;    // [N] trial / step electrode potential per node
};

// 1-D charge transport along x: line l holds the nodes off[l] .. off[l + 1] - 1 in x order
// (an x row of a regular grid or one packed column).
struct ChargeParams {
  int lines;
  const int *off;           // [lines + 1]
  double dx;                // m
  const double *iv;         // [N] A/m^3
  const double *omega;      // [N] Ohm m
  double *ia, *pel;         // [N] A/m^2, V
};

struct InitParams {
  int N, M, energy, fp32;
  double theta_ref, inv_T_ref;
  double mmin_over_m[LBM_MMAX];
  double inv_m[LBM_MMAX];
  double cv[LBM_MMAX], uf[LBM_MMAX];
  const double *X0, *Plat, *T0, *phi;
  void *pop;                // double or float (fp32)
};

// Macroscopic output set of the moments kernel: rows
//   rho_a (M), u (D), T, P, j_a (M*D), rho, X_a (M)
struct MomParams {
  KParams k;
  double *out;
};

// Mechanism of the specialised chemistry kernel (chem_jit.hip): everything that
// is written into the generated source as a literal.
struct ChemSpec {
  int M, K, R, n_sub, n_newton;
  int nu_f[LBM_RMAX][16], nu_b[LBM_RMAX][16];   // [reaction][species], species = gas, vacancy, adsorbates
  double A_f[LBM_RMAX], Ea_f[LBM_RMAX], A_b[LBM_RMAX], Ea_b[LBM_RMAX];
  double m[LBM_MMAX];                            // gas molar masses, kg/mol
  double R_U;
  int perm[16];                                  // elimination order of the S = M + K unknowns
  int kind[LBM_RMAX];                            // 0 surface, 1 homogeneous, 2 TPB edge
  double w_r[LBM_RMAX];                          // gas-row weight of a surface reaction (a^(s))
  double gam_k[16], a_k[16];                     // per surface species: site density, area
  double l_tpb;
  int charge_z[LBM_RMAX];                        // electrons released by the forward reaction
  double beta_ct[LBM_RMAX];                      // symmetry factor of a charge transfer
  int has_ct;
  int occupancy;                                 // waves per SIMD the generated kernel is compiled for (1, 2)
};

// launchers (lbm_kernels.hip)
hipError_t launch_init(int dim, const InitParams &ip, hipStream_t s);
hipError_t launch_species(int dim, const KParams &p, hipStream_t s);
hipError_t launch_mixture(int dim, const KParams &p, hipStream_t s);
hipError_t launch_chem(const ChemParams &cp, hipStream_t s);
hipError_t launch_charge(const ChargeParams &q, const SecantParams *sp, hipStream_t s);   // sp: trial
hipError_t launch_secant_start(const SecantParams &sp, hipStream_t s);
hipError_t launch_surface_energy(const KParams &p, hipStream_t s);
hipError_t launch_moments(int dim, const KParams &p, double *out, hipStream_t s);
hipError_t launch_diag(int dim, int L, int Mmom, const KParams &p, const void *pop, double *partials,
                       int nblocks, hipStream_t s);
hipError_t launch_diag_totals(const double *partials, int nblocks, int W, double *totals, hipStream_t s);
int chem_supported(int M, int K);

// adjoint of the isothermal reaction-free step (lbm_adjoint.hip)
struct AdjBuffers {
  const double *lam_next;   // Lambda_{t+1} [L][Q][N] or NULL
  double *lam_cur, *lamp;   // Lambda_t, lambda'_t
  double *gbar;             // [D][N]
  double *phibar, *kfacbar; // [N]
  double *jacc;             // [N]
  double wN;                // 1 / (T m_s)
  int out_species;
};
// stage 1: lambda'_t and dJ/dG; stage 2: Lambda_t and parameter adjoints;
// stage 3: the initial-state term (k.pin = initial populations, lam_next = Lambda_1)
hipError_t launch_adjoint(int dim, const KParams &k, const AdjBuffers &b, int stage, hipStream_t s);

// specialised chemistry (chem_jit.hip)
std::string chem_specialized_source(const ChemSpec &spec);
std::string chem_node_source(const ChemSpec &spec);
void chem_choose_order(ChemSpec &spec, int ns, const double *T, const double *phi, const double *C, double h,
                       double a_s, double gam);
hipError_t chem_specialize(const ChemSpec &spec, hipFunction_t *fn, std::string *log);
hipError_t launch_chem_specialized(hipFunction_t fn, const ChemParams &cp, hipStream_t s);

// Fused multi-step kernel for one-dimensional lattices (lbm_window.h), compiled at
// run time with the context's constants and, with a mechanism, its chemistry.
#include "lbm_window_args.h"

struct WindowSpec {
  int M, faradaic, knudsen, need_v, bc_lo, bc_hi;
  int steps;                // whole steps per launch (odd)
  int wpb;                  // waves per block
  double theta_ref, inv_T_ref, nu;
  double mmin_over_m[LBM_MMAX], inv_m[LBM_MMAX], imD[LBM_MMAX * LBM_MMAX];
  InletState inlet[2];
};
constexpr int kWindowMaxSteps = 7;   // 64 - 4 * 7 = 36 nodes per window at the most
std::string window_program_source(const ChemSpec *chem, const WindowSpec &w);
hipError_t window_specialize(const ChemSpec *chem, const WindowSpec &w, hipFunction_t *fn, std::string *log);
hipError_t launch_window(hipFunction_t fn, const WinArgs &a, int blocks, int wpb, hipStream_t s);
