// Host side of the C ABI declared in include/lbm.h: validation, the lattice
// unit system, device allocations, the per-step launch sequence, moments,
// diagnostics, timing and snapshots.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

#include <cmath>

namespace {

constexpr double kRU = 8.314462618;      // J/(mol K)
constexpr double kFC = 96485.33212;      // C/mol
constexpr int kTimingRing = 64;          // steps of per-kernel events kept

struct Buf {
  double *p = nullptr;
  size_t n = 0;
};

}  // namespace

struct lbm_ctx {
  // configuration
  int dim, nx, ny, nz, N, M, L, Q, energy, bc_lo, bc_hi;
  int n_cols;
  hipStream_t stream;
  double dx, T_ref, P_ref, theta_ref, nu, prandtl;
  double m[LBM_MMAX], m_min;
  double Dref[LBM_MMAX * LBM_MMAX];
  double cv_lat[LBM_MMAX], uf_lat[LBM_MMAX];
  double c2, dt, rho_unit;
  InletState inlet[2];
  bool have_inlet[2];
  // device buffers
  double *pop[2] = {nullptr, nullptr};   // raw storage: double, or float when fp32
  int fp32 = 0;                           // populations stored as float
  double *phi = nullptr, *kfac = nullptr, *Tfield = nullptr;
  double *X0 = nullptr, *Plat = nullptr;
  int8_t *colflag = nullptr;
  double *rA = nullptr, *rRT = nullptr, *rFk = nullptr, *rrho = nullptr, *rY = nullptr, *rqd = nullptr;
  double *rec[2] = {nullptr, nullptr};   // node records: velocity + species source
  double *T[2] = {nullptr, nullptr};
  double *srcsum = nullptr;
  double *theta = nullptr;
  double *rEs = nullptr;                  // [N] adsorbed-phase energy before the chemistry
  int esrc = 0;                           // adsorbed-phase thermo given (energy lattice)
  double es_u[LBM_KMAX] = {}, es_c[LBM_KMAX] = {};
  double *faradaic = nullptr;
  double *macro = nullptr;
  double *partials = nullptr;
  int diag_blocks = 0;
  // state
  int cur = 0;
  int first_step = 1;
  long long steps_done = 0;
  int knudsen = 0;
  double pore_radius = 0.0;
  int has_mech = 0, has_faradaic = 0;
  int has_ct = 0;                       // the mechanism has charge-transfer reactions
  int electrode = 0;                    // charge transport along x (lbm_set_electrode)
  int n_lines = 0;                      // x lines: ny nz rows of a grid, or the packed columns
  std::vector<int> line_off;            // [n_lines + 1] first node of each line
  int *d_line_off = nullptr;
  double *iv = nullptr, *ia = nullptr, *pel = nullptr, *ped = nullptr, *omega_n = nullptr;
  double *uel = nullptr;                // [N] electrical energy source (energy lattice on)
  // current control: per-line target I^(a) and secant state, trial buffers [N]
  int n_secant = 0;
  double *d_phi_line = nullptr, *d_target = nullptr, *d_p0 = nullptr, *d_f0 = nullptr, *d_p1 = nullptr;
  double *iv_try = nullptr, *ia_try = nullptr, *pel_try = nullptr, *ped_try = nullptr;
  double a_el = 0.0;                    // specific area of the electrolyte (second) surface phase
  ChemParams chem;
  ChemTables *chem_tab = nullptr;
  ChemTables chem_host;                 // host copy of the installed mechanism
  int chem_kernel = LBM_CHEM_SPECIALIZED;
  hipFunction_t chem_fn = nullptr;      // specialised kernel of the installed mechanism
  int chem_perm[16] = {};               // its elimination order (kept in snapshots)
  int have_perm = 0;
  // graph step loop: a captured sequence of graph_steps (even) steps, replayed
  int graph_steps = 0;
  hipGraphExec_t gexec = nullptr;
  int gexec_cur = -1;                   // population buffer index the capture started from
  int gexec_q = -1;                     // record buffer parity (steps_done & 1) it started from
  hipFunction_t gexec_chem = nullptr;   // chemistry kernel the capture launched
  double *gexec_theta = nullptr;        // coverage buffer the capture started from
  hipFunction_t gexec_win = nullptr;    // fused kernel the capture launched
  // fused multi-step launch of 1-D lattices (lbm_set_persistent)
  int win_steps = 0;                    // whole steps per launch (odd), 0: off
  int win_wpb = 1;                      // waves per block
  hipFunction_t win_fn = nullptr;       // compiled for the set-up in win_key
  long long win_key[8] = {};
  double *theta_alt = nullptr;          // second coverage buffer: a launch reads one, writes the other
  double *win_sk = nullptr;             // rate constants per wave and lane
  size_t win_sk_n = 0;
  size_t adj_budget = 0;                // adjoint workspace budget in bytes (0: 3/4 of free memory)
  int tile_polls = 1 << 18;             // bound of the species kernel's tile-barrier waits
  int K = 0;
  // timing
  int timing = 0;
  hipEvent_t ev[kTimingRing][5];
  int ev_count = 0;
  int ev_ready = 0;
  double t_total_ms = 0.0;
  hipEvent_t ev_all[2];
  char err[512];
};

namespace {

int fail(lbm_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, LBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

// Doubles of storage for one population field (L Q N values, 4 or 8 bytes each).
size_t pop_words(const lbm_ctx *c) {
  const size_t n = (size_t)c->L * c->Q * c->N;
  return c->fp32 ? (n + 1) / 2 : n;
}

int dalloc(lbm_ctx *c, double **p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void **)p, n * sizeof(double));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, LBM_ENOMEM, "hipMalloc of %zu doubles failed: %s", n, hipGetErrorString(e));
  }
  return LBM_OK;
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

// Equilibrium state of an inlet mixture (X, P, T) in lattice units.
InletState make_inlet(const lbm_ctx *c, const double *X, double P_Pa, double T_K) {
  InletState s;
  memset(&s, 0, sizeof(s));
  const double Pl = P_Pa / c->P_ref;
  double rho = 0.0;
  for (int a = 0; a < c->M; ++a) {
    s.RaT[a] = c->theta_ref * (c->m_min / c->m[a]) * (T_K / c->T_ref);
    s.rho_a[a] = X[a] * Pl / s.RaT[a];
    rho += s.rho_a[a];
  }
  s.rho = rho;
  double RT = 0.0, U = 0.0;
  for (int a = 0; a < c->M; ++a) {
    const double Y = s.rho_a[a] / rho;
    RT += Y * s.RaT[a];
    U += Y * (c->uf_lat[a] + c->cv_lat[a] * T_K);
  }
  s.RT = RT;
  s.U = U;
  s.T_K = T_K;
  return s;
}

KParams base_params(const lbm_ctx *c) {
  KParams p;
  memset(&p, 0, sizeof(p));
  p.N = c->N;
  p.nx = c->nx;
  p.ny = c->ny;
  p.nz = c->nz;
  p.M = c->M;
  p.energy = c->energy;
  p.bc_lo = c->bc_lo;
  p.bc_hi = c->bc_hi;
  p.knudsen = c->knudsen;
  p.colflag = c->colflag;
  p.fp32 = c->fp32;
  p.tile_polls = c->tile_polls;
  p.theta_ref = c->theta_ref;
  p.inv_T_ref = 1.0 / c->T_ref;
  p.nu = c->nu;
  p.prandtl = c->prandtl;
  for (int a = 0; a < c->M; ++a) {
    p.mmin_over_m[a] = c->m_min / c->m[a];
    p.inv_m[a] = 1.0 / c->m[a];
    p.cv[a] = c->cv_lat[a];
    p.uf[a] = c->uf_lat[a];
  }
  memcpy(p.Dref, c->Dref, sizeof(p.Dref));
  for (int a = 0; a < c->M; ++a)
    for (int b = 0; b < c->M; ++b) p.imD[a * LBM_MMAX + b] = (1.0 / c->m[b]) / c->Dref[a * LBM_MMAX + b];
  p.inlet[0] = c->inlet[0];
  p.inlet[1] = c->inlet[1];
  p.phi = c->phi;
  p.kfac = c->kfac;
  p.Tfield = c->Tfield;
  p.rA = c->rA;
  p.rRT = c->rRT;
  p.rFk = c->rFk;
  p.rrho = c->rrho;
  p.rY = c->rY;
  p.rqd = c->rqd;
  p.K = c->has_mech ? c->K : 0;
  p.esrc = c->esrc;
  p.theta = c->theta;
  p.rEs = c->rEs;
  memcpy(p.es_u, c->es_u, sizeof(p.es_u));
  memcpy(p.es_c, c->es_c, sizeof(p.es_c));
  return p;
}

// The last completed step wrote species sources into its records that the
// stored populations do not hold yet: every pull of a species lattice adds
// them.  Records of steps without chemistry hold zero sources; freshly built
// populations (first_step) have none to take.
int src_pending(const lbm_ctx *c) {
  return (c->has_mech || c->has_faradaic) && !c->first_step ? 1 : 0;
}

bool needs_v(const lbm_ctx *c) {
  return c->has_mech || c->has_faradaic || c->bc_lo == BC_INLET || c->bc_hi == BC_INLET;
}

// Parameters for reading the state at the current time level (the pull of the
// next step): records of the last completed step.
void fill_prev(const lbm_ctx *c, KParams &p) {
  const int q_last = (int)((c->steps_done + 1) & 1);   // parity of the last completed step
  p.pin = c->pop[c->cur];
  p.first_step = c->first_step;
  p.src_prev = src_pending(c);
  p.rec_prev = c->rec[q_last];
  p.T_prev = c->energy ? c->T[q_last] : c->Tfield;
}

int rebuild_populations(lbm_ctx *c) {
  InitParams ip;
  memset(&ip, 0, sizeof(ip));
  ip.N = c->N;
  ip.M = c->M;
  ip.energy = c->energy;
  ip.theta_ref = c->theta_ref;
  ip.inv_T_ref = 1.0 / c->T_ref;
  for (int a = 0; a < c->M; ++a) {
    ip.mmin_over_m[a] = c->m_min / c->m[a];
    ip.inv_m[a] = 1.0 / c->m[a];
    ip.cv[a] = c->cv_lat[a];
    ip.uf[a] = c->uf_lat[a];
  }
  ip.X0 = c->X0;
  ip.Plat = c->Plat;
  ip.T0 = c->Tfield;
  ip.phi = c->phi;
  ip.pop = c->pop[0];
  ip.fp32 = c->fp32;
  HIPCHK(c, launch_init(c->dim, ip, c->stream));
  c->cur = 0;
  c->first_step = 1;
  c->steps_done = 0;
  return LBM_OK;
}

int check_config(const lbm_config *cfg, lbm_ctx *c) {
  if (!cfg) return LBM_EINVAL;
  if (cfg->dim < 1 || cfg->dim > 3) return fail(c, LBM_EINVAL, "dim must be 1, 2 or 3");
  if (cfg->n_species < 2 || cfg->n_species > LBM_MMAX)
    return fail(c, LBM_EINVAL, "n_species must be in [2, %d]", LBM_MMAX);
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return fail(c, LBM_EINVAL, "grid extents must be >= 1");
  if ((cfg->dim < 2 && cfg->ny != 1) || (cfg->dim < 3 && cfg->nz != 1))
    return fail(c, LBM_EINVAL, "unused grid extents must be 1");
  if ((cfg->bc_lo_x == LBM_BC_PERIODIC) != (cfg->bc_hi_x == LBM_BC_PERIODIC))
    return fail(c, LBM_EINVAL, "periodic x must be set on both ends");
  for (int s = 0; s < 2; ++s) {
    const int k = s ? cfg->bc_hi_x : cfg->bc_lo_x;
    if (k < 0 || k > 3) return fail(c, LBM_EINVAL, "unknown boundary kind %d", k);
    if (k == LBM_BC_INLET && !(s ? cfg->inlet_hi_X : cfg->inlet_lo_X))
      return fail(c, LBM_EINVAL, "inlet boundary needs its mole fractions");
  }
  if (!cfg->molar_mass || !cfg->D_ref_lat) return fail(c, LBM_EINVAL, "molar_mass and D_ref_lat are required");
  if (cfg->energy_on && (!cfg->cv || !cfg->u_form)) return fail(c, LBM_EINVAL, "energy lattice needs cv and u_form");
  if (cfg->precision != LBM_FP64 && cfg->precision != LBM_FP32)
    return fail(c, LBM_EINVAL, "precision must be LBM_FP64 or LBM_FP32");
  if (!(cfg->dx_m > 0) || !(cfg->T_ref_K > 0) || !(cfg->P_ref_Pa > 0) || !(cfg->theta_ref > 0) ||
      !(cfg->theta_ref <= 1.0) || !(cfg->nu_lat > 0) || !(cfg->prandtl > 0))
    return fail(c, LBM_EINVAL, "dx, T_ref, P_ref, theta_ref in (0,1], nu and Pr must be positive");
  const int M = cfg->n_species;
  for (int a = 0; a < M; ++a)
    if (!(cfg->molar_mass[a] > 0)) return fail(c, LBM_EINVAL, "molar masses must be positive");
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b)
      if (a != b) {
        const double d = cfg->D_ref_lat[a * M + b];
        if (!(d > 0) || fabs(d - cfg->D_ref_lat[b * M + a]) > 1e-12 * d)
          return fail(c, LBM_EINVAL, "D_ref_lat must be positive and symmetric");
      }
  return LBM_OK;
}

// ---- file-scope scratch of lbm_get_diagnostics_static -------------------------
// The partial sums and totals of the no-allocation diagnostics live in this array:
// one copy on every GPU the library runs on, held until the process ends.  In host
// code its name is only a stand-in; the device address of each GPU's copy is taken
// once per device at set-up (hipGetSymbolAddress with that device current) and used
// wherever host code passes the array on.
constexpr size_t kScratchDoubles = size_t(1) << 18;   // 2 MiB
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
double *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// Address of this device's scratch copy, set up on first use per device (called
// from the init calls, with the context's device current).
int setup_scratch(lbm_ctx *c) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, LBM_EINVAL, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return LBM_OK;
}

int common_init(const lbm_config *cfg, int N, const double *X0, const double *P0, const double *T0,
                lbm_ctx *c) {
  c->dim = cfg->dim;
  c->N = N;
  c->M = cfg->n_species;
  c->energy = cfg->energy_on ? 1 : 0;
  c->fp32 = cfg->precision == LBM_FP32 ? 1 : 0;
  c->L = c->M + 1 + c->energy;
  c->Q = cfg->dim == 1 ? 3 : (cfg->dim == 2 ? 9 : 27);
  c->bc_lo = cfg->bc_lo_x;
  c->bc_hi = cfg->bc_hi_x;
  c->stream = (hipStream_t)cfg->hip_stream;
  c->dx = cfg->dx_m;
  c->T_ref = cfg->T_ref_K;
  c->P_ref = cfg->P_ref_Pa;
  c->theta_ref = cfg->theta_ref;
  c->nu = cfg->nu_lat;
  c->prandtl = cfg->prandtl;
  c->m_min = 1e300;
  memset(c->Dref, 0, sizeof(c->Dref));
  for (int a = 0; a < c->M; ++a) {
    c->m[a] = cfg->molar_mass[a];
    c->m_min = fmin(c->m_min, c->m[a]);
    for (int b = 0; b < c->M; ++b) c->Dref[a * LBM_MMAX + b] = (a == b) ? 1.0 : cfg->D_ref_lat[a * c->M + b];
  }
  // lattice unit system: R T of the lightest species at T_ref equals theta_ref
  c->c2 = kRU * c->T_ref / (c->m_min * c->theta_ref);
  c->dt = c->dx / sqrt(c->c2);
  c->rho_unit = c->P_ref / c->c2;
  for (int a = 0; a < c->M; ++a) {
    c->cv_lat[a] = c->energy ? cfg->cv[a] / c->c2 : 0.0;
    c->uf_lat[a] = c->energy ? cfg->u_form[a] / c->c2 : 0.0;
  }
  // host-side validation of the fields
  if (!X0 || !T0) return fail(c, LBM_EINVAL, "X0 and T0 are required");
  double Tmax = 0.0;
  for (int n = 0; n < N; ++n) {
    double sx = 0.0;
    for (int a = 0; a < c->M; ++a) {
      const double x = X0[(size_t)a * N + n];
      if (!(x >= 0.0)) return fail(c, LBM_EINVAL, "negative mole fraction at node %d", n);
      sx += x;
    }
    if (fabs(sx - 1.0) > 1e-9) return fail(c, LBM_EINVAL, "mole fractions at node %d sum to %.17g", n, sx);
    if (!(T0[n] > 0)) return fail(c, LBM_EINVAL, "temperature must be positive");
    if (P0 && !(P0[n] > 0)) return fail(c, LBM_EINVAL, "pressure must be positive");
    Tmax = fmax(Tmax, T0[n]);
  }
  // positivity of the product form at rest: the lightest species R T <= 1
  if (c->theta_ref * Tmax / c->T_ref > 1.0) return fail(c, LBM_EINVAL, "R_a T exceeds 1 (product form not positive)");
  for (int s = 0; s < 2; ++s) {
    const double *X = s ? cfg->inlet_hi_X : cfg->inlet_lo_X;
    c->have_inlet[s] = X != nullptr;
    if (X) {
      double sx = 0.0;
      for (int a = 0; a < c->M; ++a) sx += X[a];
      if (fabs(sx - 1.0) > 1e-9 || !(cfg->inlet_P_Pa > 0) || !(cfg->inlet_T_K > 0))
        return fail(c, LBM_EINVAL, "inlet state invalid");
      if (c->theta_ref * cfg->inlet_T_K / c->T_ref > 1.0) return fail(c, LBM_EINVAL, "inlet R_a T exceeds 1");
      c->inlet[s] = make_inlet(c, X, cfg->inlet_P_Pa, cfg->inlet_T_K);
    } else {
      memset(&c->inlet[s], 0, sizeof(InletState));
    }
  }
  // device allocations
  const size_t popn = pop_words(c);
  int rc;
  if ((rc = dalloc(c, &c->pop[0], popn)) || (rc = dalloc(c, &c->pop[1], popn))) return rc;
  if ((rc = dalloc(c, &c->phi, N)) || (rc = dalloc(c, &c->kfac, N)) || (rc = dalloc(c, &c->Tfield, N)) ||
      (rc = dalloc(c, &c->X0, (size_t)c->M * N)) || (rc = dalloc(c, &c->Plat, N)))
    return rc;
  const int D = c->dim;
  if ((rc = dalloc(c, &c->rA, (size_t)D * N)) || (rc = dalloc(c, &c->rRT, N)) ||
      (rc = dalloc(c, &c->rFk, (size_t)D * N)) || (rc = dalloc(c, &c->rrho, (size_t)c->M * N)) ||
      (rc = dalloc(c, &c->rec[0], (size_t)kRec * N)) || (rc = dalloc(c, &c->rec[1], (size_t)kRec * N)) ||
      (rc = dalloc(c, &c->srcsum, N)))
    return rc;
  if (c->energy) {
    if ((rc = dalloc(c, &c->rY, (size_t)(c->M + 2) * N)) || (rc = dalloc(c, &c->rqd, (size_t)D * N)) ||
        (rc = dalloc(c, &c->T[0], N)) || (rc = dalloc(c, &c->T[1], N)))
      return rc;
  }
  const size_t mrows = (size_t)(c->M + D + 2 + c->M * D + 1 + c->M);
  if ((rc = dalloc(c, &c->macro, mrows * N))) return rc;
  c->diag_blocks = (N + 255) / 256;
  if ((rc = dalloc(c, &c->partials, (size_t)c->diag_blocks * (c->L + D + 2)))) return rc;
  // upload fields
  std::vector<double> Plat(N), ones(N, 1.0), zeros((size_t)kRec * N, 0.0);
  for (int n = 0; n < N; ++n) Plat[n] = (P0 ? P0[n] : c->P_ref) / c->P_ref;
  HIPCHK(c, hipMemcpy(c->X0, X0, sizeof(double) * c->M * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->Plat, Plat.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->Tfield, T0, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->phi, ones.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->kfac, zeros.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->rec[0], zeros.data(), sizeof(double) * kRec * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->rec[1], zeros.data(), sizeof(double) * kRec * N, hipMemcpyHostToDevice));
  if (c->energy) {
    HIPCHK(c, hipMemcpy(c->T[0], T0, sizeof(double) * N, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->T[1], T0, sizeof(double) * N, hipMemcpyHostToDevice));
  }
  c->knudsen = 0;
  memset(&c->chem, 0, sizeof(c->chem));
  rc = rebuild_populations(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return setup_scratch(c);
}

int sample_order(lbm_ctx *c, ChemSpec &sp);

// Builds the mechanism-specialised chemistry kernel.  The elimination order is
// chosen on Newton matrices sampled (up to 64 nodes spread over the grid) from
// the chemistry input and coverages of the last step, so it is called after a
// first step has run with the generic kernel; compilation happens once per
// mechanism and process.
// Mechanism of the context as written into generated code (elimination order
// excluded).
void fill_chem_spec(const lbm_ctx *c, ChemSpec &sp) {
  const int M = c->M, K = c->K, S = M + K;
  const ChemParams &cp = c->chem;
  memset(&sp, 0, sizeof(sp));
  sp.M = M;
  sp.K = K;
  sp.R = cp.R;
  sp.n_sub = cp.n_sub;
  sp.n_newton = cp.n_newton;
  for (int r = 0; r < cp.R; ++r) {
    for (int t = 0; t < S; ++t) {
      sp.nu_f[r][t] = c->chem_host.nu_f[r][t];
      sp.nu_b[r][t] = c->chem_host.nu_b[r][t];
    }
    sp.A_f[r] = c->chem_host.A_f[r];
    sp.Ea_f[r] = c->chem_host.Ea_f[r];
    sp.A_b[r] = c->chem_host.A_b[r];
    sp.Ea_b[r] = c->chem_host.Ea_b[r];
    sp.kind[r] = c->chem_host.kind[r];
    sp.w_r[r] = c->chem_host.w_r[r];
    sp.charge_z[r] = c->chem_host.charge_z[r];
    sp.beta_ct[r] = c->chem_host.beta_ct[r];
  }
  sp.has_ct = c->has_ct;
  for (int a = 0; a < M; ++a) sp.m[a] = c->m[a];
  for (int k = 0; k < K; ++k) {
    sp.gam_k[k] = c->chem_host.gam_k[k];
    sp.a_k[k] = c->chem_host.a_k[k];
  }
  sp.l_tpb = c->chem_host.l_tpb;
  sp.R_U = kRU;
}

int specialize_chemistry(lbm_ctx *c) {
  ChemSpec sp;
  fill_chem_spec(c, sp);
  sp.occupancy = c->chem_kernel == LBM_CHEM_SPECIALIZED_2W ? 2 : 1;
  if (c->have_perm) {
    memcpy(sp.perm, c->chem_perm, sizeof(sp.perm));
  } else {
    const int rc = sample_order(c, sp);
    if (rc) return rc;
  }
  std::string log;
  const hipError_t e = chem_specialize(sp, &c->chem_fn, &log);
  if (e != hipSuccess) {
    c->chem_fn = nullptr;
    return fail(c, LBM_EHIP, "specialised chemistry kernel: %s (%s)", hipGetErrorString(e), log.c_str());
  }
  memcpy(c->chem_perm, sp.perm, sizeof(sp.perm));
  c->have_perm = 1;
  return LBM_OK;
}

// Elimination order from Newton matrices at up to 64 sampled nodes.
int sample_order(lbm_ctx *c, ChemSpec &sp) {
  const int M = c->M, K = c->K, S = M + K, N = c->N;
  const ChemParams &cp = c->chem;
  const int ns = N < 64 ? N : 64;
  std::vector<double> T(ns), phi(ns), C((size_t)ns * S);
  const double *Tsrc = c->energy ? c->T[(c->steps_done + 1) & 1] : c->Tfield;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int j = 0; j < ns; ++j) {
    const size_t n = (size_t)j * N / ns;
    double x;
    HIPCHK(c, hipMemcpy(&T[j], Tsrc + n, sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&phi[j], c->phi + n, sizeof(double), hipMemcpyDeviceToHost));
    for (int a = 0; a < M; ++a) {
      HIPCHK(c, hipMemcpy(&x, c->rrho + (size_t)a * N + n, sizeof(double), hipMemcpyDeviceToHost));
      C[(size_t)j * S + a] = x * c->rho_unit / c->m[a];
    }
    for (int k = 0; k < K; ++k) {
      HIPCHK(c, hipMemcpy(&x, c->theta + (size_t)k * N + n, sizeof(double), hipMemcpyDeviceToHost));
      C[(size_t)j * S + M + k] = sp.gam_k[k] * x;
    }
  }
  chem_choose_order(sp, ns, T.data(), phi.data(), C.data(), c->dt / cp.n_sub, cp.a_s, cp.gamma);
  return LBM_OK;
}

int enqueue_step(lbm_ctx *c, int record_slot) {
  const int q = (int)(c->steps_done & 1);
  KParams p = base_params(c);
  p.pin = c->pop[c->cur];
  p.pout = c->pop[1 - c->cur];
  p.first_step = c->first_step;
  const int chem = c->has_mech || c->has_faradaic;
  p.chem = chem;
  p.need_v = needs_v(c) ? 1 : 0;
  p.src_prev = src_pending(c);
  p.rec_prev = c->rec[1 - q];
  p.rec_cur = c->rec[q];
  p.T_prev = c->energy ? c->T[1 - q] : c->Tfield;
  p.T_cur = c->energy ? c->T[q] : nullptr;
  p.srcsum_cur = c->srcsum;
  const bool elec_energy = c->energy && c->electrode && c->has_ct;
  p.uel = elec_energy ? c->uel : nullptr;
  hipEvent_t *ev = record_slot >= 0 ? c->ev[record_slot] : nullptr;
  if (ev) HIPCHK(c, hipEventRecord(ev[0], c->stream));
  HIPCHK(c, launch_species(c->dim, p, c->stream));
  if (ev) HIPCHK(c, hipEventRecord(ev[1], c->stream));
  if (p.esrc) HIPCHK(c, launch_surface_energy(p, c->stream));   // before the coverages change
  if (chem) {
    ChemParams cp = c->chem;
    cp.N = c->N;
    cp.M = c->M;
    cp.K = c->has_mech ? c->K : 0;
    cp.rrho = c->rrho;
    cp.T = c->energy ? c->T[q] : c->Tfield;
    cp.phi = c->phi;
    cp.faradaic = c->has_faradaic ? c->faradaic : nullptr;
    cp.theta = c->theta;
    cp.rec = c->rec[q];
    cp.srcsum = c->srcsum;
    cp.dt = c->dt;
    cp.rho_unit = c->rho_unit;
    cp.R_U = kRU;
    cp.F_C = kFC;
    cp.iv = c->has_ct ? c->iv : nullptr;
    cp.pel = c->electrode ? c->pel : nullptr;
    cp.ped = c->electrode ? c->ped : nullptr;
    cp.uel = elec_energy ? c->uel : nullptr;
    cp.omega = c->omega_n;
    cp.a_el = c->a_el;
    cp.dx = c->dx;
    cp.inv_e_unit = 1.0 / (c->rho_unit * c->c2);
    for (int a = 0; a < c->M; ++a) cp.m[a] = c->m[a];
    if (c->n_secant && c->electrode && c->has_ct) {   // current control before the step's chemistry
      ChemParams tp = cp;
      tp.dry = 1;
      tp.ped = c->ped_try;
      tp.iv = c->iv_try;
      tp.uel = nullptr;
      ChargeParams tq;
      tq.lines = c->n_lines;
      tq.off = c->d_line_off;
      tq.dx = c->dx;
      tq.iv = c->iv_try;
      tq.omega = c->omega_n;
      tq.ia = c->ia_try;
      tq.pel = c->pel_try;
      SecantParams sp;
      sp.lines = c->n_lines;
      sp.off = c->d_line_off;
      sp.ia = c->ia_try;
      sp.target = c->d_target;
      sp.p0 = c->d_p0;
      sp.f0 = c->d_f0;
      sp.p1 = c->d_p1;
      sp.phi_line = c->d_phi_line;
      sp.ped_try = c->ped_try;
      sp.ped = c->ped;
      sp.stage = 0;
      sp.final_iter = 0;
      HIPCHK(c, launch_secant_start(sp, c->stream));
      for (int it = 0; it <= c->n_secant; ++it) {
        if (c->chem_fn)
          HIPCHK(c, launch_chem_specialized(c->chem_fn, tp, c->stream));
        else
          HIPCHK(c, launch_chem(tp, c->stream));
        sp.stage = it == 0 ? 0 : 1;
        sp.final_iter = it == c->n_secant ? 1 : 0;
        HIPCHK(c, launch_charge(tq, &sp, c->stream));   // integrates the trial and takes the secant step
      }
    }
    if (c->chem_fn)
      HIPCHK(c, launch_chem_specialized(c->chem_fn, cp, c->stream));
    else
      HIPCHK(c, launch_chem(cp, c->stream));
  }
  if (c->electrode) {           // the next step's rates see the potentials of this step's currents
    ChargeParams q;
    q.lines = c->n_lines;
    q.off = c->d_line_off;
    q.dx = c->dx;
    q.iv = c->iv;
    q.omega = c->omega_n;
    q.ia = c->ia;
    q.pel = c->pel;
    HIPCHK(c, launch_charge(q, nullptr, c->stream));
  }
  if (ev) HIPCHK(c, hipEventRecord(ev[2], c->stream));
  if (ev) HIPCHK(c, hipEventRecord(ev[3], c->stream));   // no separate source pass (added at the pull)
  HIPCHK(c, launch_mixture(c->dim, p, c->stream));
  if (ev) HIPCHK(c, hipEventRecord(ev[4], c->stream));
  c->cur = 1 - c->cur;
  c->first_step = 0;
  c->steps_done += 1;
  return LBM_OK;
}

// Whether the fused 1-D kernel covers this context: D1Q3, isothermal, FP64
// populations, non-periodic x ends, and either the specialised chemistry of a
// mechanism (with or without a Faradaic source) or no chemistry at all, no
// electrode coupling.  Returns a reason when it does not.
const char *window_unsupported(const lbm_ctx *c) {
  if (c->dim != 1) return "the fused kernel is for one-dimensional lattices";
  if (c->energy) return "the fused kernel has no energy lattice";
  if (c->fp32) return "the fused kernel stores FP64 populations";
  if (c->bc_lo == BC_PERIODIC || c->bc_hi == BC_PERIODIC) return "the fused kernel needs closed x ends";
  if (c->electrode || c->n_secant) return "the fused kernel has no electrode coupling";
  if (c->has_faradaic && !c->has_mech) return "a Faradaic source without a mechanism runs the separate kernels";
  if (c->has_mech && c->chem_kernel == LBM_CHEM_GENERIC) return "the fused kernel takes the specialised chemistry";
  return nullptr;
}

// A launch can start here: past the first step, the chemistry specialised.
bool window_ready(const lbm_ctx *c) {
  if (!c->win_steps || c->first_step || c->steps_done < 1 || window_unsupported(c)) return false;
  if (c->has_mech && (!c->chem_fn || !c->have_perm)) return false;
  return true;
}

int window_blocks(const lbm_ctx *c, int steps, int wpb) {
  const int use = 64 - 4 * steps;
  const int waves = (c->N + use - 1) / use;
  return (waves + wpb - 1) / wpb;
}

// Compiles the fused kernel for the current configuration and sizes its buffers.
int window_prepare(lbm_ctx *c) {
  // what the generated source depends on beyond the constants fixed at init
  const long long key[8] = {c->win_steps, c->win_wpb, c->has_mech, c->has_faradaic, c->knudsen,
                            needs_v(c) ? 1 : 0, (long long)(intptr_t)c->chem_fn, c->K};
  if (c->win_fn && memcmp(key, c->win_key, sizeof(key)) == 0) return LBM_OK;
  WindowSpec w;
  memset(&w, 0, sizeof(w));
  const KParams p = base_params(c);
  w.M = c->M;
  w.faradaic = c->has_faradaic;
  w.knudsen = c->knudsen;
  w.need_v = needs_v(c) ? 1 : 0;
  w.bc_lo = c->bc_lo;
  w.bc_hi = c->bc_hi;
  w.steps = c->win_steps;
  w.wpb = c->win_wpb;
  w.theta_ref = p.theta_ref;
  w.inv_T_ref = p.inv_T_ref;
  w.nu = p.nu;
  memcpy(w.mmin_over_m, p.mmin_over_m, sizeof(w.mmin_over_m));
  memcpy(w.inv_m, p.inv_m, sizeof(w.inv_m));
  memcpy(w.imD, p.imD, sizeof(w.imD));
  w.inlet[0] = c->inlet[0];
  w.inlet[1] = c->inlet[1];
  ChemSpec sp;
  if (c->has_mech) {
    fill_chem_spec(c, sp);
    memcpy(sp.perm, c->chem_perm, sizeof(sp.perm));
    const size_t need = (size_t)window_blocks(c, c->win_steps, c->win_wpb) * c->win_wpb * 2 * c->chem.R * 64;
    if (need > c->win_sk_n) {
      dfree(c->win_sk);
      c->win_sk = nullptr;
      c->win_sk_n = 0;
      const int rc = dalloc(c, &c->win_sk, need);
      if (rc) return rc;
      c->win_sk_n = need;
    }
    if (!c->theta_alt) {
      const int rc = dalloc(c, &c->theta_alt, (size_t)c->K * c->N);
      if (rc) return rc;
    }
  }
  std::string log;
  hipFunction_t fn = nullptr;
  const hipError_t e = window_specialize(c->has_mech ? &sp : nullptr, w, &fn, &log);
  if (e != hipSuccess) return fail(c, LBM_EHIP, "fused 1-D kernel: %s (%s)", hipGetErrorString(e), log.c_str());
  c->win_fn = fn;
  memcpy(c->win_key, key, sizeof(key));
  return LBM_OK;
}

// One launch of win_steps whole steps (an odd count: the populations and the
// node records land in the buffers the last of that many separate steps would
// write, the coverages in the other coverage buffer).
int enqueue_window(lbm_ctx *c) {
  const int rc = window_prepare(c);
  if (rc) return rc;
  if (!c->win_fn || (c->has_mech && (!c->theta || !c->theta_alt || !c->win_sk)))
    return fail(c, LBM_ESTATE, "fused 1-D kernel: buffers missing");
  const int q = (int)(c->steps_done & 1);
  WinArgs a;
  memset(&a, 0, sizeof(a));
  a.N = c->N;
  a.nx = c->colflag ? 0 : c->nx;
  a.colflag = reinterpret_cast<const signed char *>(c->colflag);
  a.pin = c->pop[c->cur];
  a.pout = c->pop[1 - c->cur];
  a.rec_prev = c->rec[1 - q];
  a.rec_out = c->rec[q];
  a.phi = c->phi;
  a.kfac = c->kfac;
  a.Tf = c->Tfield;
  a.far = c->has_faradaic ? c->faradaic : nullptr;
  a.theta_in = c->theta;
  a.theta_out = c->theta_alt;
  a.rrho = c->rrho;
  a.rRT = c->rRT;
  a.rA = c->rA;
  a.rFk = c->rFk;
  a.srcsum = c->srcsum;
  a.skg = c->win_sk;
  a.dt = c->dt;
  a.rho_unit = c->rho_unit;
  a.fuel = c->chem.fuel;
  a.product = c->chem.product;
  HIPCHK(c, launch_window(c->win_fn, a, window_blocks(c, c->win_steps, c->win_wpb), c->win_wpb, c->stream));
  c->cur = 1 - c->cur;
  c->first_step = 0;
  c->steps_done += c->win_steps;
  if (c->has_mech) std::swap(c->theta, c->theta_alt);
  return LBM_OK;
}

// Steps of one graph replay: graph_steps, or with the fused kernel the next
// multiple of twice its steps per launch (every buffer back where it started).
int graph_len(const lbm_ctx *c) {
  if (!c->win_steps) return c->graph_steps;
  const int two = 2 * c->win_steps;
  return (c->graph_steps + two - 1) / two * two;
}

void drop_graph(lbm_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gexec_cur = -1;
  c->gexec_q = -1;
  c->gexec_chem = nullptr;
  c->gexec_theta = nullptr;
  c->gexec_win = nullptr;
}

// Captures graph_steps steps starting from the current state into c->gexec.
// Nothing runs during the capture; the context's step state is restored after it.
int capture_steps(lbm_ctx *c) {
  drop_graph(c);
  const int cur0 = c->cur, first0 = c->first_step;
  const long long done0 = c->steps_done;
  if (c->win_steps) {                   // compile and size the buffers before the capture
    const int rc0 = window_prepare(c);
    if (rc0) return rc0;
  }
  double *theta0 = c->theta, *theta_alt0 = c->theta_alt;   // the launches swap them
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = LBM_OK;
  const int len = graph_len(c);
  for (int s = 0; s < len && rc == LBM_OK;) {
    if (window_ready(c) && len - s >= c->win_steps) {
      rc = enqueue_window(c);
      s += c->win_steps;
    } else {
      rc = enqueue_step(c, -1);
      ++s;
    }
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->cur = cur0;
  c->first_step = first0;
  c->steps_done = done0;
  c->theta = theta0;
  c->theta_alt = theta_alt0;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return fail(c, LBM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->gexec = nullptr;
    return fail(c, LBM_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
  }
  c->gexec_cur = cur0;
  c->gexec_q = (int)(done0 & 1);
  c->gexec_chem = c->chem_fn;
  c->gexec_theta = theta0;
  c->gexec_win = c->win_fn;
  return LBM_OK;
}

// Steady state for the graph: past the first (identity-pull) step and with the
// chemistry kernel of the remaining run in place.
bool graph_ready(const lbm_ctx *c) {
  if (!c->graph_steps || c->first_step || c->steps_done < 1) return false;
  if (c->has_mech && c->chem_kernel != LBM_CHEM_GENERIC && !c->chem_fn) return false;
  return true;
}

}  // namespace

extern "C" {

int lbm_init(const lbm_config *cfg, const double *X0, const double *P0, const double *T0, lbm_ctx **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->err[0] = 0;
  int rc = check_config(cfg, c);
  if (rc) {
    *out = c;   // caller can read the message, then destroy
    return rc;
  }
  c->nx = cfg->nx;
  c->ny = cfg->ny;
  c->nz = cfg->nz;
  c->n_cols = 0;
  rc = common_init(cfg, cfg->nx * cfg->ny * cfg->nz, X0, P0, T0, c);
  *out = c;
  return rc;
}

int lbm_init_columns(const lbm_config *cfg, int32_t n_cols, const int32_t *col_len, const double *X0,
                     const double *P0, const double *T0, lbm_ctx **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->err[0] = 0;
  *out = c;
  int rc = check_config(cfg, c);
  if (rc) return rc;
  if (cfg->dim != 1) return fail(c, LBM_EINVAL, "packed columns need dim == 1");
  if (cfg->bc_lo_x == LBM_BC_PERIODIC) return fail(c, LBM_EINVAL, "packed columns cannot be periodic");
  if (n_cols < 1 || !col_len) return fail(c, LBM_EINVAL, "need at least one column");
  long long N = 0;
  for (int k = 0; k < n_cols; ++k) {
    if (col_len[k] < 2) return fail(c, LBM_EINVAL, "columns need at least 2 nodes");
    N += col_len[k];
  }
  if (N > (1LL << 30)) return fail(c, LBM_EINVAL, "too many nodes");
  c->nx = (int)N;
  c->ny = c->nz = 1;
  c->n_cols = n_cols;
  c->line_off.assign(n_cols + 1, 0);
  for (int k = 0; k < n_cols; ++k) c->line_off[k + 1] = c->line_off[k] + col_len[k];
  rc = common_init(cfg, (int)N, X0, P0, T0, c);
  if (rc) return rc;
  std::vector<int8_t> flag(N, 0);
  long long o = 0;
  for (int k = 0; k < n_cols; ++k) {
    flag[o] |= 1;
    flag[o + col_len[k] - 1] |= 2;
    o += col_len[k];
  }
  hipError_t e = hipMalloc((void **)&c->colflag, N);
  if (e != hipSuccess) return fail(c, LBM_ENOMEM, "hipMalloc colflag");
  HIPCHK(c, hipMemcpy(c->colflag, flag.data(), N, hipMemcpyHostToDevice));
  return LBM_OK;
}

int lbm_set_porous_field(lbm_ctx *c, const double *phi, const double *tort, double pore_radius_m) {
  if (!c) return LBM_EINVAL;
  if (c->steps_done) return fail(c, LBM_ESTATE, "lbm_set_porous_field after the first step");
  if (!phi) return fail(c, LBM_EINVAL, "phi is required");
  const int N = c->N;
  const bool kn = pore_radius_m > 0.0 && isfinite(pore_radius_m);
  std::vector<double> kf(N, 0.0);
  const double pref = kn ? (2.0 * pore_radius_m / (3.0 * c->dx)) * sqrt(8.0 / M_PI) : 0.0;
  for (int n = 0; n < N; ++n) {
    if (!(phi[n] > 0.0 && phi[n] <= 1.0)) return fail(c, LBM_EINVAL, "porosity at node %d not in (0,1]", n);
    const double t = tort ? tort[n] : 1.0;
    if (!(t > 0.0)) return fail(c, LBM_EINVAL, "tortuosity must be positive");
    kf[n] = kn ? (phi[n] / t) * pref : 0.0;
  }
  HIPCHK(c, hipMemcpy(c->phi, phi, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->kfac, kf.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  c->knudsen = kn ? 1 : 0;
  c->pore_radius = pore_radius_m;
  int rc = rebuild_populations(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_set_mechanism(lbm_ctx *c, const lbm_mechanism *mech) {
  if (!c) return LBM_EINVAL;
  if (c->steps_done) return fail(c, LBM_ESTATE, "lbm_set_mechanism after the first step");
  if (!mech) {
    c->has_mech = 0;
    c->has_ct = 0;
    c->K = 0;
    c->esrc = 0;
    return LBM_OK;
  }
  const int M = c->M, K = mech->n_surface, R = mech->n_reactions, S = M + K;
  if (K < 2 || K > LBM_KMAX || R < 1 || R > LBM_RMAX) return fail(c, LBM_EINVAL, "mechanism sizes out of range");
  if (!chem_supported(M, K)) return fail(c, LBM_EINVAL, "no chemistry kernel for (M, K) = (%d, %d)", M, K);
  if (mech->n_sub < 1 || mech->n_newton < 1) return fail(c, LBM_EINVAL, "n_sub and n_newton must be >= 1");
  if (!mech->nu_f || !mech->nu_b || !mech->A_f || !mech->Ea_f || !mech->A_b || !mech->Ea_b || !mech->theta0)
    return fail(c, LBM_EINVAL, "mechanism arrays missing");
  if (!(mech->gamma > 0) || !(mech->a_s > 0)) return fail(c, LBM_EINVAL, "gamma and a_s must be positive");
  const int fuel = c->chem.fuel, product = c->chem.product;
  ChemTables tab;
  memset(&tab, 0, sizeof(tab));
  // surface phases: site density and specific area per surface species
  int phase[LBM_KMAX];
  bool two = false;
  for (int k = 0; k < K; ++k) {
    phase[k] = mech->surface_phase ? mech->surface_phase[k] : 0;
    if (phase[k] != 0 && phase[k] != 1) return fail(c, LBM_EINVAL, "surface_phase must be 0 or 1");
    two = two || phase[k] == 1;
  }
  if (two && (!(mech->gamma2 > 0) || !(mech->a_s2 > 0)))
    return fail(c, LBM_EINVAL, "a second surface phase needs gamma2 and a_s2 > 0");
  for (int k = 0; k < K; ++k) {
    tab.gam_k[k] = phase[k] ? mech->gamma2 : mech->gamma;
    tab.a_k[k] = phase[k] ? mech->a_s2 : mech->a_s;
  }
  tab.l_tpb = mech->l_tpb;
  bool has_ct = false;
  for (int r = 0; r < R; ++r) {
    int site[2][2] = {{0, 0}, {0, 0}};           // [phase][forward, backward]
    bool gas = false, ph_in[2] = {false, false};
    for (int s = 0; s < S; ++s) {
      const int ef = mech->nu_f[r * S + s], eb = mech->nu_b[r * S + s];
      if (ef < 0 || ef > 3 || eb < 0 || eb > 3) return fail(c, LBM_EINVAL, "stoichiometric coefficients must be 0..3");
      tab.nu_f[r][s] = (int8_t)ef;
      tab.nu_b[r][s] = (int8_t)eb;
      if (s >= M) {
        site[phase[s - M]][0] += ef;
        site[phase[s - M]][1] += eb;
        if (ef || eb) ph_in[phase[s - M]] = true;
      } else if (ef || eb) {
        gas = true;
      }
    }
    if (site[0][0] != site[0][1] || site[1][0] != site[1][1])
      return fail(c, LBM_EINVAL, "reaction %d is not site-balanced on every phase", r);
    const int hom = mech->homogeneous ? mech->homogeneous[r] : 0;
    const int edge = mech->edge ? mech->edge[r] : 0;
    if (hom != 0 && hom != 1) return fail(c, LBM_EINVAL, "homogeneous flags must be 0 or 1");
    if (edge != 0 && edge != 1) return fail(c, LBM_EINVAL, "edge flags must be 0 or 1");
    if (hom && edge) return fail(c, LBM_EINVAL, "reaction %d cannot be homogeneous and an edge reaction", r);
    if (hom) {                        // gas species only, zero net mass (eq sumRhoDot)
      double dm = 0.0, mm = 0.0;
      for (int s = 0; s < S; ++s) {
        const int ef = mech->nu_f[r * S + s], eb = mech->nu_b[r * S + s];
        if (s >= M && (ef || eb)) return fail(c, LBM_EINVAL, "homogeneous reaction %d has surface species", r);
        if (s < M) {
          dm += (eb - ef) * c->m[s];
          mm += (eb + ef) * c->m[s];
        }
      }
      if (fabs(dm) > 1e-12 * mm) return fail(c, LBM_EINVAL, "homogeneous reaction %d changes the mass", r);
    }
    if (edge) {                       // adsorbed species only, rate per unit TPB length
      if (gas) return fail(c, LBM_EINVAL, "edge reaction %d has gas species", r);
      if (!(mech->l_tpb > 0)) return fail(c, LBM_EINVAL, "edge reactions need l_tpb > 0");
    }
    if (!hom && !edge && ph_in[0] && ph_in[1])
      return fail(c, LBM_EINVAL, "surface reaction %d spans two phases (mark it as an edge reaction)", r);
    const int z = mech->charge_z ? mech->charge_z[r] : 0;
    if (z) {                          // charge transfer at the TPB
      if (!edge) return fail(c, LBM_EINVAL, "charge-transfer reaction %d must be a TPB edge reaction", r);
      if (z < -4 || z > 4) return fail(c, LBM_EINVAL, "reaction %d: charge_z must lie in -4..4", r);
      if (!mech->beta_ct || !(mech->beta_ct[r] >= 0.0 && mech->beta_ct[r] <= 1.0))
        return fail(c, LBM_EINVAL, "reaction %d: symmetry factor beta_ct must lie in [0, 1]", r);
      tab.beta_ct[r] = mech->beta_ct[r];
      has_ct = true;
    }
    tab.charge_z[r] = (int8_t)z;
    tab.kind[r] = (int8_t)(hom ? 1 : (edge ? 2 : 0));
    tab.w_r[r] = ph_in[1] && !ph_in[0] ? mech->a_s2 : mech->a_s;
    if (!std::isfinite(mech->A_f[r]) || !std::isfinite(mech->A_b[r]) || !std::isfinite(mech->Ea_f[r]) ||
        !std::isfinite(mech->Ea_b[r]) || mech->A_f[r] < 0 || mech->A_b[r] < 0)
      return fail(c, LBM_EINVAL, "reaction %d: pre-factors must be finite and >= 0, energies finite", r);
    tab.A_f[r] = mech->A_f[r];
    tab.Ea_f[r] = mech->Ea_f[r];
    tab.A_b[r] = mech->A_b[r];
    tab.Ea_b[r] = mech->Ea_b[r];
  }
  if (!c->chem_tab) {
    hipError_t e = hipMalloc((void **)&c->chem_tab, sizeof(ChemTables));
    if (e != hipSuccess) return fail(c, LBM_ENOMEM, "hipMalloc chemistry tables");
  }
  HIPCHK(c, hipMemcpy(c->chem_tab, &tab, sizeof(tab), hipMemcpyHostToDevice));
  c->chem_host = tab;
  c->chem_fn = nullptr;
  c->have_perm = 0;
  ChemParams &cp = c->chem;
  memset(&cp, 0, sizeof(cp));
  cp.tab = c->chem_tab;
  cp.R = R;
  cp.n_sub = mech->n_sub;
  cp.n_newton = mech->n_newton;
  cp.gamma = mech->gamma;
  cp.a_s = mech->a_s;
  cp.fuel = fuel;
  cp.product = product;
  double st[2] = {0.0, 0.0};
  for (int s = 0; s < K; ++s) st[phase[s]] += mech->theta0[s];
  if (fabs(st[0] - 1.0) > 1e-9 || (two && fabs(st[1] - 1.0) > 1e-9))
    return fail(c, LBM_EINVAL, "theta0 must sum to 1 on every surface phase");
  dfree(c->theta);
  c->theta = nullptr;
  dfree(c->theta_alt);
  c->theta_alt = nullptr;
  int rc = dalloc(c, &c->theta, (size_t)K * c->N);
  if (rc) return rc;
  std::vector<double> th((size_t)K * c->N);
  for (int s = 0; s < K; ++s)
    for (int n = 0; n < c->N; ++n) th[(size_t)s * c->N + n] = mech->theta0[s];
  HIPCHK(c, hipMemcpy(c->theta, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice));
  // adsorbed-phase internal energy per unit volume, lattice units (eq temperatureCell):
  // a_s Gamma theta_k m_k (u_form_k + cv_k T) / (rho_unit c^2)
  c->esrc = 0;
  memset(c->es_u, 0, sizeof(c->es_u));
  memset(c->es_c, 0, sizeof(c->es_c));
  if (c->energy && mech->surf_cv) {
    if (!mech->surf_mass) return fail(c, LBM_EINVAL, "adsorbed-phase thermo needs surf_mass");
    for (int k = 0; k < K; ++k) {
      const double w = tab.a_k[k] * tab.gam_k[k] * mech->surf_mass[k] / (c->rho_unit * c->c2);
      if (!std::isfinite(w) || !std::isfinite(mech->surf_cv[k]) ||
          (mech->surf_u_form && !std::isfinite(mech->surf_u_form[k])))
        return fail(c, LBM_EINVAL, "adsorbed-phase thermo must be finite");
      c->es_c[k] = w * mech->surf_cv[k];
      c->es_u[k] = mech->surf_u_form ? w * mech->surf_u_form[k] : 0.0;
    }
    if (!c->rEs) {
      const int rc2 = dalloc(c, &c->rEs, c->N);
      if (rc2) return rc2;
    }
    c->esrc = 1;
  }
  if (has_ct && !c->iv) {
    const int rc3 = dalloc(c, &c->iv, c->N);
    if (rc3) return rc3;
    HIPCHK(c, hipMemset(c->iv, 0, sizeof(double) * c->N));
  }
  c->has_ct = has_ct ? 1 : 0;
  c->a_el = mech->a_s2;
  c->K = K;
  c->has_mech = 1;
  return LBM_OK;
}

int lbm_set_electrode(lbm_ctx *c, const double *phi_electrode, const double *omega) {
  if (!c) return LBM_EINVAL;
  drop_graph(c);                // captured steps read the electrode arrays of their set-up
  if (!phi_electrode) {
    c->electrode = 0;
    return LBM_OK;
  }
  if (!omega) return fail(c, LBM_EINVAL, "omega is required with an electrode potential");
  if (c->line_off.empty()) {    // regular grid: the ny nz rows along x
    const int L = c->ny * c->nz;
    c->line_off.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) c->line_off[l + 1] = c->line_off[l] + c->nx;
  }
  const int L = (int)c->line_off.size() - 1;
  for (int l = 0; l < L; ++l)
    if (!std::isfinite(phi_electrode[l])) return fail(c, LBM_EINVAL, "electrode potential of line %d not finite", l);
  for (int n = 0; n < c->N; ++n)
    if (!std::isfinite(omega[n]) || omega[n] < 0.0)
      return fail(c, LBM_EINVAL, "resistivity omega[%d] must be finite and >= 0", n);
  if (!c->pel) {
    double **bufs[] = {&c->ia, &c->pel, &c->ped, &c->omega_n, &c->uel,
                       &c->iv_try, &c->ia_try, &c->pel_try, &c->ped_try};
    for (double **b : bufs) {
      const int rc = dalloc(c, b, c->N);
      if (rc) return rc;
      HIPCHK(c, hipMemset(*b, 0, sizeof(double) * c->N));
    }
    double **lb[] = {&c->d_phi_line, &c->d_target, &c->d_p0, &c->d_f0, &c->d_p1};
    for (double **b : lb) {
      const int rc = dalloc(c, b, L);
      if (rc) return rc;
      HIPCHK(c, hipMemset(*b, 0, sizeof(double) * L));
    }
    const hipError_t e = hipMalloc((void **)&c->d_line_off, sizeof(int) * (L + 1));
    if (e != hipSuccess) return fail(c, LBM_ENOMEM, "hipMalloc line offsets");
    HIPCHK(c, hipMemcpy(c->d_line_off, c->line_off.data(), sizeof(int) * (L + 1), hipMemcpyHostToDevice));
    c->n_lines = L;
  }
  if (!c->iv) {
    const int rc = dalloc(c, &c->iv, c->N);
    if (rc) return rc;
    HIPCHK(c, hipMemset(c->iv, 0, sizeof(double) * c->N));
  }
  std::vector<double> ped(c->N);
  for (int l = 0; l < L; ++l)
    for (int n = c->line_off[l]; n < c->line_off[l + 1]; ++n) ped[n] = phi_electrode[l];
  HIPCHK(c, hipMemcpy(c->ped, ped.data(), sizeof(double) * c->N, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_phi_line, phi_electrode, sizeof(double) * L, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->omega_n, omega, sizeof(double) * c->N, hipMemcpyHostToDevice));
  c->electrode = 1;
  return LBM_OK;
}

int lbm_set_current_target(lbm_ctx *c, const double *target_ia, int32_t n_secant) {
  if (!c) return LBM_EINVAL;
  drop_graph(c);
  if (!target_ia) {
    c->n_secant = 0;
    return LBM_OK;
  }
  if (!c->electrode || !c->has_ct)
    return fail(c, LBM_ESTATE, "current control needs an electrode and a charge-transfer mechanism");
  if (n_secant < 1 || n_secant > 64) return fail(c, LBM_EINVAL, "n_secant must lie in 1..64");
  for (int l = 0; l < c->n_lines; ++l)
    if (!std::isfinite(target_ia[l])) return fail(c, LBM_EINVAL, "target current of line %d not finite", l);
  HIPCHK(c, hipMemcpy(c->d_target, target_ia, sizeof(double) * c->n_lines, hipMemcpyHostToDevice));
  c->n_secant = n_secant;
  return LBM_OK;
}

int lbm_get_electrode_potential(lbm_ctx *c, double *phi_line) {
  if (!c || !phi_line) return LBM_EINVAL;
  if (!c->electrode) return fail(c, LBM_ESTATE, "no electrode installed");
  HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
  HIPCHK(c, hipMemcpy(phi_line, c->d_phi_line, sizeof(double) * c->n_lines, hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_get_charge(lbm_ctx *c, double *iv, double *ia, double *phi_el) {
  if (!c) return LBM_EINVAL;
  if (!c->has_ct && !c->electrode)
    return fail(c, LBM_ESTATE, "no charge-transfer mechanism and no electrode installed");
  HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
  const size_t bytes = sizeof(double) * c->N;
  double *outs[] = {iv, ia, phi_el};
  const double *srcs[] = {c->iv, c->ia, c->pel};
  for (int k = 0; k < 3; ++k) {
    if (!outs[k]) continue;
    if (srcs[k])
      HIPCHK(c, hipMemcpy(outs[k], srcs[k], bytes, hipMemcpyDeviceToHost));
    else
      memset(outs[k], 0, bytes);
  }
  return LBM_OK;
}

int lbm_set_chem_kernel(lbm_ctx *c, int32_t kind) {
  if (!c) return LBM_EINVAL;
  if (kind != LBM_CHEM_SPECIALIZED && kind != LBM_CHEM_GENERIC && kind != LBM_CHEM_SPECIALIZED_2W)
    return fail(c, LBM_EINVAL, "unknown chemistry kernel %d", kind);
  // between the two generated forms the elimination order stays: only the register budget differs
  const bool keep_order = kind != LBM_CHEM_GENERIC && c->chem_kernel != LBM_CHEM_GENERIC;
  c->chem_kernel = kind;
  c->chem_fn = nullptr;
  if (!keep_order) c->have_perm = 0;
  drop_graph(c);
  return LBM_OK;
}

int lbm_set_faradaic_source(lbm_ctx *c, const double *rate, int32_t fuel, int32_t product) {
  if (!c) return LBM_EINVAL;
  if (c->steps_done) return fail(c, LBM_ESTATE, "lbm_set_faradaic_source after the first step");
  if (!rate) {
    c->has_faradaic = 0;
    return LBM_OK;
  }
  if (fuel < 0 || fuel >= c->M || product < 0 || product >= c->M || fuel == product)
    return fail(c, LBM_EINVAL, "fuel/product species out of range");
  if (!c->faradaic) {
    int rc = dalloc(c, &c->faradaic, c->N);
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpy(c->faradaic, rate, sizeof(double) * c->N, hipMemcpyHostToDevice));
  c->chem.fuel = fuel;
  c->chem.product = product;
  c->has_faradaic = 1;
  return LBM_OK;
}

int lbm_set_graph(lbm_ctx *c, int32_t steps_per_graph) {
  if (!c) return LBM_EINVAL;
  if (steps_per_graph != 0 && (steps_per_graph < 2 || steps_per_graph % 2))
    return fail(c, LBM_EINVAL, "steps_per_graph must be 0 or an even number >= 2");
  if (steps_per_graph && !c->stream) return fail(c, LBM_EINVAL, "the graph step loop needs a non-null stream");
  c->graph_steps = steps_per_graph;
  drop_graph(c);
  return LBM_OK;
}

int lbm_set_persistent(lbm_ctx *c, int32_t steps_per_launch, int32_t waves_per_block) {
  if (!c) return LBM_EINVAL;
  if (steps_per_launch == 0) {
    c->win_steps = 0;
    drop_graph(c);
    return LBM_OK;
  }
  if (steps_per_launch < 1 || steps_per_launch > kWindowMaxSteps || steps_per_launch % 2 == 0)
    return fail(c, LBM_EINVAL, "steps_per_launch must be 0 or odd, 1..%d", kWindowMaxSteps);
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(c, LBM_EINVAL, "waves_per_block must be 1, 2 or 4");
  const char *why = window_unsupported(c);
  if (why) return fail(c, LBM_EINVAL, "%s", why);
  c->win_steps = steps_per_launch;
  c->win_wpb = waves_per_block;
  drop_graph(c);
  return LBM_OK;
}

int lbm_autotune(lbm_ctx *c, int32_t trial_steps, lbm_tune_entry *table, int32_t max_entries,
                 int32_t *n_entries) {
  if (!c || !n_entries || (max_entries > 0 && !table)) return LBM_EINVAL;
  if (trial_steps < 2) return fail(c, LBM_EINVAL, "trial_steps must be >= 2");
  if (c->steps_done < 1 || c->first_step) return fail(c, LBM_ESTATE, "lbm_autotune needs a completed first step");
  if (!c->stream) return fail(c, LBM_EINVAL, "lbm_autotune needs a non-null stream");
  // candidates: the separate kernels (plain launches, graph of 32 steps) and,
  // where it applies, the fused kernel at 1, 3, 5 steps per launch and 1 or 2
  // waves per block
  std::vector<lbm_tune_entry> cand;   // {fused, chem_kernel, graph_steps, steps_per_launch, waves_per_block, ms}
  const int chem0 = c->chem_kernel;
  const int gen = chem0 == LBM_CHEM_GENERIC ? LBM_CHEM_GENERIC : LBM_CHEM_SPECIALIZED;
  cand.push_back({0, gen, 0, 0, 0, 0.0});
  cand.push_back({0, gen, 32, 0, 0, 0.0});
  if (c->has_mech && gen == LBM_CHEM_SPECIALIZED) cand.push_back({0, LBM_CHEM_SPECIALIZED_2W, 32, 0, 0, 0.0});
  if (!window_unsupported(c))
    for (int st : {1, 3, 5})
      for (int wpb : {1, 2}) cand.push_back({1, gen, 0, st, wpb, 0.0});
  size_t snap_n = 0;
  int rc = lbm_save(c, nullptr, &snap_n);
  if (rc) return rc;
  std::vector<char> snap(snap_n);
  rc = lbm_save(c, snap.data(), &snap_n);
  if (rc) return rc;
  const int graph0 = c->graph_steps, win0 = c->win_steps, wpb0 = c->win_wpb, timing0 = c->timing;
  c->timing = 0;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  int best = -1;
  for (size_t k = 0; k < cand.size() && rc == LBM_OK; ++k) {
    lbm_tune_entry &t = cand[k];
    rc = lbm_load(c, snap.data(), snap_n);
    if (rc) break;
    c->graph_steps = t.graph_steps;
    c->win_steps = t.steps_per_launch;
    c->win_wpb = t.waves_per_block ? t.waves_per_block : 1;
    if (c->has_mech && t.chem_kernel != c->chem_kernel) {   // the other generated form, same order
      c->chem_kernel = t.chem_kernel;
      c->chem_fn = nullptr;
    }
    drop_graph(c);
    // whole launches or graph replays only: a multiple of 2 x steps per launch
    const int unit = t.graph_steps ? graph_len(c) : (t.steps_per_launch ? 2 * t.steps_per_launch : 2);
    const int n = (trial_steps + unit - 1) / unit * unit;
    rc = lbm_step(c, unit);                  // compiles and captures outside the timed steps
    if (rc) break;
    HIPCHK(c, hipEventRecord(e0, c->stream));
    rc = lbm_step(c, n);
    if (rc) break;
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    t.ms_per_step = (double)ms / n;
    if (best < 0 || t.ms_per_step < cand[best].ms_per_step) best = (int)k;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = timing0;
  const int rcl = lbm_load(c, snap.data(), snap_n);
  if (rc || rcl || best < 0) {
    c->graph_steps = graph0;
    c->win_steps = win0;
    c->win_wpb = wpb0;
    if (c->chem_kernel != chem0) {
      c->chem_kernel = chem0;
      c->chem_fn = nullptr;
    }
    drop_graph(c);
    return rc ? rc : (rcl ? rcl : fail(c, LBM_EHIP, "no candidate measured"));
  }
  c->graph_steps = cand[best].graph_steps;
  c->win_steps = cand[best].steps_per_launch;
  c->win_wpb = cand[best].waves_per_block ? cand[best].waves_per_block : 1;
  if (c->chem_kernel != cand[best].chem_kernel) {
    c->chem_kernel = cand[best].chem_kernel;
    c->chem_fn = nullptr;
  }
  drop_graph(c);
  *n_entries = (int32_t)cand.size();
  for (int k = 0; k < (int)cand.size() && k < max_entries; ++k) table[k] = cand[k];
  return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t n_steps) {
  if (!c) return LBM_EINVAL;
  if (n_steps < 0) return fail(c, LBM_EINVAL, "negative step count");

  if (c->timing) {
    HIPCHK(c, hipEventRecord(c->ev_all[0], c->stream));
  }
  const int64_t first_timed = n_steps > kTimingRing ? n_steps - kTimingRing : 0;
  int slot = 0;
  for (int64_t s = 0; s < n_steps;) {
    if (c->has_mech && c->chem_kernel != LBM_CHEM_GENERIC && !c->chem_fn && c->steps_done >= 1) {
      const int rc = specialize_chemistry(c);   // after the first step (generic kernel)
      if (rc) return rc;
    }
    // graph replay: whole captured sequences from the parity the capture started at
    const int len = graph_len(c);
    if (graph_ready(c) && n_steps - s >= len &&
        (!c->gexec || (c->gexec_cur == c->cur && c->gexec_q == (int)(c->steps_done & 1) &&
                       c->gexec_theta == c->theta))) {
      if (!c->gexec || c->gexec_chem != c->chem_fn || (c->win_steps && c->gexec_win != c->win_fn)) {
        const int rc = capture_steps(c);
        if (rc) return rc;
      }
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->steps_done += len;                     // an even count: the buffer parity is unchanged
      s += len;
      continue;
    }
    if (window_ready(c) && n_steps - s >= c->win_steps) {   // fused launch of several steps
      const int rc = enqueue_window(c);
      if (rc) return rc;
      s += c->win_steps;
      continue;
    }
    const int rec = (c->timing && s >= first_timed) ? slot++ : -1;
    int rc = enqueue_step(c, rec);
    if (rc) return rc;
    ++s;
  }
  if (c->timing) {
    HIPCHK(c, hipEventRecord(c->ev_all[1], c->stream));
    c->ev_count = slot;
    c->ev_ready = 1;
  }
  return LBM_OK;
}

int lbm_adjoint_outlet_flux(lbm_ctx *c, int64_t n_steps, int32_t species, double *J, double *grad_phi,
                            double *grad_rp, int32_t out_on_device) {
  if (!c || !J || !grad_phi || !grad_rp) return LBM_EINVAL;
  if (n_steps < 1) return fail(c, LBM_EINVAL, "n_steps must be >= 1");
  if (species < 0 || species >= c->M) return fail(c, LBM_EINVAL, "species out of range");
  if (c->energy || c->has_mech || c->has_faradaic || c->colflag || c->fp32)
    return fail(c, LBM_EINVAL, "the adjoint covers isothermal, reaction-free grids with FP64 storage");
  if (c->steps_done != 0) return fail(c, LBM_ESTATE, "the adjoint starts from the initial state (no step taken)");
  const size_t N = c->N, L = c->L, Q = c->Q, D = c->dim;
  const size_t P = L * Q * N, R = (size_t)kRec * N, A = D * N;
  const int64_t T = n_steps;
  // Segments of K steps, the last one ending at T; every state of a segment is kept
  // in slots while its adjoint runs.  The forward pass checkpoints the start of every
  // segment but the last, whose steps it computes straight into the slots, so the
  // forward work is 2 T - K: K as large as the workspace budget allows (K = T: a
  // single segment, nothing recomputed).
  const size_t slot = P + R + A, ckw = P + R, fixed = 3 * P + A + 3 * N;
  size_t budget = c->adj_budget;
  if (!budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
    budget = fr / 4 * 3;
  }
  auto need_of = [&](int64_t k) {
    const int64_t ns = (T + k - 1) / k;
    return sizeof(double) * ((size_t)(ns - 1) * ckw + (size_t)(k + 1) * slot + fixed);
  };
  int64_t K = 0;                                      // the largest that fits
  size_t least = (size_t)-1;
  for (int64_t k = T; k >= 1 && !K; --k) {
    const size_t nk = need_of(k);
    if (nk <= budget) K = k;
    least = nk < least ? nk : least;
  }
  if (!K)
    return fail(c, LBM_ENOMEM, "adjoint workspace of at least %.2f GB exceeds the budget of %.2f GB", least / 1e9,
                budget / 1e9);
  const int64_t nseg = (T + K - 1) / K;
  auto seg_end = [&](int64_t s) { return T - (nseg - 1 - s) * K; };
  auto seg_start = [&](int64_t s) { return seg_end(s) - K > 0 ? seg_end(s) - K : 0; };
  const size_t need = need_of(K) / sizeof(double);
  double *ws = nullptr;
  if (hipMalloc((void **)&ws, sizeof(double) * need) != hipSuccess)
    return fail(c, LBM_ENOMEM, "adjoint workspace of %.2f GB", 8.0 * need / 1e9);
  double *ck = ws;                                    // [nseg - 1][P + R]
  double *seg = ck + (size_t)(nseg - 1) * ckw;        // [K + 1][P + R + A]
  double *lam[2] = {seg + (size_t)(K + 1) * slot, nullptr};
  lam[1] = lam[0] + P;
  double *lamp = lam[1] + P, *gbar = lamp + P, *phibar = gbar + A, *kfacbar = phibar + N, *jacc = kfacbar + N;
  auto slot_pop = [&](int64_t k) { return seg + (size_t)k * slot; };
  auto slot_rec = [&](int64_t k) { return slot_pop(k) + P; };
  auto slot_rA = [&](int64_t k) { return slot_pop(k) + P + R; };
  int rc = LBM_OK;
  double *pop0 = c->pop[0], *pop1 = c->pop[1], *rec0 = c->rec[0], *rec1 = c->rec[1], *rA0 = c->rA;
  auto restore_ptrs = [&]() {
    c->pop[0] = pop0;
    c->pop[1] = pop1;
    c->rec[0] = rec0;
    c->rec[1] = rec1;
    c->rA = rA0;
  };
  auto hipck = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && rc == LBM_OK) rc = fail(c, LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return e == hipSuccess;
  };
  // steps t0 + 1 .. t1 from the state in slot 0, step t writing slot t - t0
  auto run_into_slots = [&](int64_t t0, int64_t t1) {
    c->steps_done = t0;
    c->first_step = t0 == 0;
    c->cur = 0;
    for (int64_t t = t0 + 1; t <= t1 && rc == LBM_OK; ++t) {
      const int64_t k = t - t0 - 1;
      const int q = (int)(c->steps_done & 1);
      c->pop[c->cur] = slot_pop(k);
      c->pop[1 - c->cur] = slot_pop(k + 1);
      c->rec[1 - q] = slot_rec(k);
      c->rec[q] = slot_rec(k + 1);
      c->rA = slot_rA(k);
      rc = enqueue_step(c, -1);
    }
    restore_ptrs();
  };
  hipck(hipMemsetAsync(lam[0], 0, sizeof(double) * (3 * P + A + 3 * N), c->stream), "clear");
  // forward pass: checkpoints at the start of every segment but the last
  for (int64_t s = 0; s + 1 < nseg && rc == LBM_OK; ++s) {
    const int q_last = (int)((c->steps_done + 1) & 1);
    hipck(hipMemcpyAsync(ck + (size_t)s * ckw, c->pop[c->cur], sizeof(double) * P, hipMemcpyDeviceToDevice,
                         c->stream), "checkpoint");
    hipck(hipMemcpyAsync(ck + (size_t)s * ckw + P, c->rec[q_last], sizeof(double) * R, hipMemcpyDeviceToDevice,
                         c->stream), "checkpoint");
    for (int64_t t = seg_start(s); t < seg_end(s) && rc == LBM_OK; ++t) rc = enqueue_step(c, -1);
  }
  // ... and the last segment straight into the slots; the state at T goes back to
  // the context's own buffers
  if (rc == LBM_OK) {
    const int q_last = (int)((c->steps_done + 1) & 1);
    hipck(hipMemcpyAsync(slot_pop(0), c->pop[c->cur], sizeof(double) * P, hipMemcpyDeviceToDevice, c->stream),
          "segment start");
    hipck(hipMemcpyAsync(slot_rec(0), c->rec[q_last], sizeof(double) * R, hipMemcpyDeviceToDevice, c->stream),
          "segment start");
    run_into_slots(seg_start(nseg - 1), T);
    const int q_T = (int)((T + 1) & 1);
    hipck(hipMemcpyAsync(c->pop[0], slot_pop(K), sizeof(double) * P, hipMemcpyDeviceToDevice, c->stream), "state");
    hipck(hipMemcpyAsync(c->rec[q_T], slot_rec(K), sizeof(double) * R, hipMemcpyDeviceToDevice, c->stream), "state");
    c->cur = 0;
    c->steps_done = T;
    c->first_step = 0;
  }
  const int cur_f = c->cur, first_f = c->first_step;
  const long long done_f = c->steps_done;
  const double wN = 1.0 / ((double)T * c->m[species]);
  // reverse sweep, segment by segment (the last one is already in the slots)
  for (int64_t s = nseg - 1; s >= 0 && rc == LBM_OK; --s) {
    const int64_t t0 = seg_start(s), t1 = seg_end(s);
    if (s + 1 < nseg) {                               // recompute the segment from its checkpoint
      hipck(hipMemcpyAsync(slot_pop(0), ck + (size_t)s * ckw, sizeof(double) * ckw, hipMemcpyDeviceToDevice,
                           c->stream), "restore");
      run_into_slots(t0, t1);
    }
    // adjoint of the segment's steps, last first
    for (int64_t t = t1; t > t0 && rc == LBM_OK; --t) {
      const int64_t k = t - t0 - 1;
      KParams ka = base_params(c);
      ka.pin = slot_pop(k);
      ka.rec_prev = slot_rec(k);
      ka.rA = slot_rA(k);
      ka.first_step = t == 1;
      AdjBuffers b;
      b.lam_next = t == T ? nullptr : lam[(t + 1) & 1];
      b.lam_cur = lam[t & 1];
      b.lamp = lamp;
      b.gbar = gbar;
      b.phibar = phibar;
      b.kfacbar = kfacbar;
      b.jacc = jacc;
      b.wN = wN;
      b.out_species = species;
      hipck(launch_adjoint(c->dim, ka, b, 1, c->stream), "adjoint pass 1");
      hipck(launch_adjoint(c->dim, ka, b, 2, c->stream), "adjoint pass 2");
    }
  }
  restore_ptrs();
  if (rc == LBM_OK) {
    KParams ka = base_params(c);
    ka.pin = slot_pop(0);                             // initial populations (slot 0 of the first segment)
    AdjBuffers b;
    memset(&b, 0, sizeof(b));
    b.lam_next = lam[1];                              // Lambda_1
    b.phibar = phibar;
    hipck(launch_adjoint(c->dim, ka, b, 3, c->stream), "adjoint initial state");
  }
  c->cur = cur_f;
  c->first_step = first_f;
  c->steps_done = done_f;
  if (rc == LBM_OK) {
    std::vector<double> hb(3 * N), kf(N), ph(N);
    hipck(hipStreamSynchronize(c->stream), "synchronize");
    hipck(hipMemcpy(hb.data(), phibar, sizeof(double) * 3 * N, hipMemcpyDeviceToHost), "copy");
    hipck(hipMemcpy(kf.data(), c->kfac, sizeof(double) * N, hipMemcpyDeviceToHost), "copy");
    hipck(hipMemcpy(ph.data(), c->phi, sizeof(double) * N, hipMemcpyDeviceToHost), "copy");
    double jsum = 0.0, rsum = 0.0;
    std::vector<double> g(N);
    for (size_t n = 0; n < N; ++n) {
      const double kb = hb[N + n];
      const double dkf = c->knudsen ? kb * kf[n] : 0.0;   // kfac is proportional to phi and to r_p
      g[n] = hb[n] + dkf / ph[n];
      rsum += dkf;
      jsum += hb[2 * N + n];
    }
    *J = jsum;
    *grad_rp = c->knudsen && c->pore_radius > 0 ? rsum / c->pore_radius : 0.0;
    hipck(hipMemcpy(grad_phi, g.data(), sizeof(double) * N,
                    out_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost), "copy gradient");
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(ws);
  return rc;
}

int lbm_set_tile_wait_limit(lbm_ctx *c, int32_t polls) {
  if (!c) return LBM_EINVAL;
  if (polls < 0) return fail(c, LBM_EINVAL, "polls must be >= 0");
  c->tile_polls = polls;
  drop_graph(c);
  return LBM_OK;
}

int lbm_set_adjoint_memory(lbm_ctx *c, uint64_t bytes) {
  if (!c) return LBM_EINVAL;
  c->adj_budget = (size_t)bytes;
  return LBM_OK;
}

int lbm_moment_rows(const lbm_ctx *c, uint32_t mask, int32_t *rows) {
  if (!c || !rows) return LBM_EINVAL;
  const int M = c->M, D = c->dim;
  int r = 0;
  if (mask & LBM_MOM_RHO_SPECIES) r += M;
  if (mask & LBM_MOM_VELOCITY) r += D;
  if (mask & LBM_MOM_TEMPERATURE) r += 1;
  if (mask & LBM_MOM_PRESSURE) r += 1;
  if (mask & LBM_MOM_SPECIES_FLUX) r += M * D;
  if (mask & LBM_MOM_COVERAGE) r += c->has_mech ? c->K : 0;
  if (mask & LBM_MOM_DENSITY) r += 1;
  if (mask & LBM_MOM_MOLE_FRACTION) r += M;
  *rows = r;
  return LBM_OK;
}

int lbm_moments(lbm_ctx *c, uint32_t mask, double *out, int32_t out_on_device) {
  if (!c) return LBM_EINVAL;
  if (!mask || !out) return fail(c, LBM_EINVAL, "empty mask or NULL output");
  KParams p = base_params(c);
  fill_prev(c, p);
  HIPCHK(c, launch_moments(c->dim, p, c->macro, c->stream));
  const int M = c->M, D = c->dim, N = c->N;
  const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  size_t o = 0;
  auto copy_rows = [&](size_t row0, size_t nrows, const double *base) -> int {
    HIPCHK(c, hipMemcpyAsync(out + o * N, base + row0 * N, sizeof(double) * nrows * N, kind, c->stream));
    o += nrows;
    return LBM_OK;
  };
  const size_t r_rho = 0, r_u = M, r_T = M + D, r_P = M + D + 1, r_j = M + D + 2, r_rhom = M + D + 2 + M * D,
               r_X = r_rhom + 1;
  int rc = LBM_OK;
  if (mask & LBM_MOM_RHO_SPECIES) rc |= copy_rows(r_rho, M, c->macro);
  if (mask & LBM_MOM_VELOCITY) rc |= copy_rows(r_u, D, c->macro);
  if (mask & LBM_MOM_TEMPERATURE) rc |= copy_rows(r_T, 1, c->macro);
  if (mask & LBM_MOM_PRESSURE) rc |= copy_rows(r_P, 1, c->macro);
  if (mask & LBM_MOM_SPECIES_FLUX) rc |= copy_rows(r_j, (size_t)M * D, c->macro);
  if ((mask & LBM_MOM_COVERAGE) && c->has_mech) rc |= copy_rows(0, c->K, c->theta);
  if (mask & LBM_MOM_DENSITY) rc |= copy_rows(r_rhom, 1, c->macro);
  if (mask & LBM_MOM_MOLE_FRACTION) rc |= copy_rows(r_X, M, c->macro);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_get_diagnostics(lbm_ctx *c, lbm_diag *out) {
  if (!c || !out) return LBM_EINVAL;
  memset(out, 0, sizeof(*out));
  const int W = c->L + c->dim + 2;
  KParams p = base_params(c);
  fill_prev(c, p);
  HIPCHK(c, launch_diag(c->dim, c->L, c->M, p, c->pop[c->cur], c->partials, c->diag_blocks, c->stream));
  std::vector<double> h((size_t)c->diag_blocks * W);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->partials, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double mn = INFINITY, bad = 0.0;
  for (int b = 0; b < c->diag_blocks; ++b) {
    const double *r = &h[(size_t)b * W];
    for (int a = 0; a < c->M && a < 8; ++a) out->species_mass[a] += r[a];
    out->mixture_mass += r[c->M];
    if (c->energy) out->energy_total += r[c->M + 1];
    for (int d = 0; d < c->dim; ++d) out->mixture_momentum[d] += r[c->L + d];
    mn = fmin(mn, r[c->L + c->dim]);
    bad += r[c->L + c->dim + 1];
  }
  out->min_population = mn;
  out->n_nonfinite = (int64_t)bad;
  out->steps_done = c->steps_done;
  if (bad > 0) return fail(c, LBM_EUNSTABLE, "%lld non-finite populations", (long long)bad);
  return LBM_OK;
}

int lbm_get_diagnostics_static(lbm_ctx *c, lbm_diag *out) {
  if (!c || !out) return LBM_EINVAL;
  memset(out, 0, sizeof(*out));
  const int W = c->L + c->dim + 2;
  const size_t need = (size_t)c->diag_blocks * W + W;
  if (need > kScratchDoubles)
    return fail(c, LBM_EINVAL, "lbm_get_diagnostics_static needs %zu doubles of scratch for %d nodes; "
                "the static buffer holds %zu (at most about %zu nodes for this lattice set)",
                need, c->N, kScratchDoubles, (kScratchDoubles - W) / W * 256);
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  double *ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
  if (!ptr) return fail(c, LBM_ESTATE, "no static scratch set up on device %d (create a context there first)", dev);
  KParams p = base_params(c);
  fill_prev(c, p);
  // every block writes all W of its partials and the totals pass writes all W
  // totals, so nothing in the array has to start at zero
  double *partials = ptr, *totals = ptr + (size_t)c->diag_blocks * W;
  HIPCHK(c, launch_diag(c->dim, c->L, c->M, p, c->pop[c->cur], partials, c->diag_blocks, c->stream));
  HIPCHK(c, launch_diag_totals(partials, c->diag_blocks, W, totals, c->stream));
  double t[64];
  HIPCHK(c, hipMemcpyAsync(t, totals, sizeof(double) * W, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int a = 0; a < c->M && a < 8; ++a) out->species_mass[a] = t[a];
  out->mixture_mass = t[c->M];
  if (c->energy) out->energy_total = t[c->M + 1];
  for (int d = 0; d < c->dim; ++d) out->mixture_momentum[d] = t[c->L + d];
  out->min_population = t[c->L + c->dim];
  const double bad = t[c->L + c->dim + 1];
  out->n_nonfinite = (int64_t)bad;
  out->steps_done = c->steps_done;
  if (bad > 0) return fail(c, LBM_EUNSTABLE, "%lld non-finite populations", (long long)bad);
  return LBM_OK;
}

int lbm_set_timing(lbm_ctx *c, int32_t enable) {
  if (!c) return LBM_EINVAL;
  if (enable && !c->timing) {
    for (int s = 0; s < kTimingRing; ++s)
      for (int k = 0; k < 5; ++k) HIPCHK(c, hipEventCreate(&c->ev[s][k]));
    HIPCHK(c, hipEventCreate(&c->ev_all[0]));
    HIPCHK(c, hipEventCreate(&c->ev_all[1]));
    c->timing = 1;
  } else if (!enable && c->timing) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < kTimingRing; ++s)
      for (int k = 0; k < 5; ++k) (void)hipEventDestroy(c->ev[s][k]);
    (void)hipEventDestroy(c->ev_all[0]);
    (void)hipEventDestroy(c->ev_all[1]);
    c->timing = 0;
  }
  c->ev_ready = 0;
  return LBM_OK;
}

int lbm_get_timing(lbm_ctx *c, double *total_ms, double *species_ms, double *chem_ms, double *mixture_ms) {
  if (!c) return LBM_EINVAL;
  if (!c->timing || !c->ev_ready || c->ev_count == 0) return fail(c, LBM_ESTATE, "no timed step recorded");
  HIPCHK(c, hipEventSynchronize(c->ev_all[1]));
  float t = 0.f;
  HIPCHK(c, hipEventElapsedTime(&t, c->ev_all[0], c->ev_all[1]));
  double acc[4] = {0, 0, 0, 0};
  for (int s = 0; s < c->ev_count; ++s)
    for (int k = 0; k < 4; ++k) {
      float e = 0;
      HIPCHK(c, hipEventElapsedTime(&e, c->ev[s][k], c->ev[s][k + 1]));
      acc[k] += e;
    }
  if (total_ms) *total_ms = t;
  if (species_ms) *species_ms = acc[0] / c->ev_count;
  if (chem_ms) *chem_ms = acc[1] / c->ev_count;
  if (mixture_ms) *mixture_ms = (acc[2] + acc[3]) / c->ev_count;   // chemistry end to mixture end
  return LBM_OK;
}

namespace {
struct SnapHeader {
  uint64_t magic, N, L, Q, M, K, D;
  int64_t steps_done;
  int32_t first_step, have_perm, fp32, electrode;
  int32_t perm[16];          // elimination order of the specialised chemistry kernel
};
constexpr uint64_t kMagic = 0x324d424c5844ull;
}  // namespace

int lbm_save(lbm_ctx *c, void *buf, size_t *size) {
  if (!c || !size) return LBM_EINVAL;
  const size_t N = c->N, D = c->dim, M = c->M;
  const size_t npop = pop_words(c);
  const size_t nrec = (size_t)kRec * N + (c->energy ? N : 0) + (c->has_mech ? (size_t)c->K * N : 0);
  // electrode state: electrolyte potential, currents, electrode potential per node and per line
  const size_t nel = c->electrode ? 4 * N + (size_t)c->n_lines : 0;
  const size_t need = sizeof(SnapHeader) + sizeof(double) * (npop + nrec + nel);
  if (!buf) {
    *size = need;
    return LBM_OK;
  }
  if (*size < need) return fail(c, LBM_EINVAL, "snapshot buffer too small (%zu < %zu)", *size, need);
  SnapHeader h;
  memset(&h, 0, sizeof(h));
  h.magic = kMagic;
  h.N = N;
  h.L = (uint64_t)c->L;
  h.Q = (uint64_t)c->Q;
  h.M = M;
  h.K = (uint64_t)c->K;
  h.D = D;
  h.steps_done = c->steps_done;
  h.first_step = c->first_step;
  h.have_perm = c->have_perm;
  h.fp32 = c->fp32;
  h.electrode = c->electrode;
  memcpy(h.perm, c->chem_perm, sizeof(h.perm));
  memcpy(buf, &h, sizeof(h));
  double *o = (double *)((char *)buf + sizeof(h));
  const int q_last = (int)((c->steps_done + 1) & 1);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(o, c->pop[c->cur], sizeof(double) * npop, hipMemcpyDeviceToHost));
  o += npop;
  HIPCHK(c, hipMemcpy(o, c->rec[q_last], sizeof(double) * kRec * N, hipMemcpyDeviceToHost));
  o += (size_t)kRec * N;
  if (c->energy) {
    HIPCHK(c, hipMemcpy(o, c->T[q_last], sizeof(double) * N, hipMemcpyDeviceToHost));
    o += N;
  }
  if (c->has_mech) {
    HIPCHK(c, hipMemcpy(o, c->theta, sizeof(double) * c->K * N, hipMemcpyDeviceToHost));
    o += (size_t)c->K * N;
  }
  if (c->electrode) {
    const double *src[] = {c->pel, c->iv, c->ia, c->ped};
    for (const double *s : src) {
      HIPCHK(c, hipMemcpy(o, s, sizeof(double) * N, hipMemcpyDeviceToHost));
      o += N;
    }
    HIPCHK(c, hipMemcpy(o, c->d_phi_line, sizeof(double) * c->n_lines, hipMemcpyDeviceToHost));
  }
  *size = need;
  return LBM_OK;
}

int lbm_load(lbm_ctx *c, const void *buf, size_t size) {
  if (!c || !buf || size < sizeof(SnapHeader)) return LBM_EINVAL;
  SnapHeader h;
  memcpy(&h, buf, sizeof(h));
  const size_t N = c->N, D = c->dim, M = c->M;
  if (h.magic != kMagic || h.N != N || h.L != (uint64_t)c->L || h.Q != (uint64_t)c->Q || h.M != M ||
      h.D != D || h.K != (uint64_t)c->K || h.fp32 != c->fp32)
    return fail(c, LBM_EINVAL, "snapshot does not match this context");
  if (h.electrode != c->electrode)
    return fail(c, LBM_EINVAL, "snapshot and context differ in the electrode coupling (install it before loading)");
  const size_t npop = pop_words(c);
  const size_t nrec = (size_t)kRec * N + (c->energy ? N : 0) + (c->has_mech ? (size_t)c->K * N : 0);
  const size_t nel = c->electrode ? 4 * N + (size_t)c->n_lines : 0;
  if (size < sizeof(SnapHeader) + sizeof(double) * (npop + nrec + nel))
    return fail(c, LBM_EINVAL, "snapshot truncated");
  drop_graph(c);
  c->steps_done = h.steps_done;
  c->first_step = h.first_step;
  if (h.have_perm && c->have_perm && memcmp(h.perm, c->chem_perm, sizeof(h.perm)) != 0) c->chem_fn = nullptr;
  c->have_perm = h.have_perm;
  memcpy(c->chem_perm, h.perm, sizeof(h.perm));
  if (!h.have_perm) c->chem_fn = nullptr;
  c->cur = 0;
  const int q_last = (int)((c->steps_done + 1) & 1);
  const double *o = (const double *)((const char *)buf + sizeof(h));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->pop[0], o, sizeof(double) * npop, hipMemcpyHostToDevice));
  o += npop;
  HIPCHK(c, hipMemcpy(c->rec[q_last], o, sizeof(double) * kRec * N, hipMemcpyHostToDevice));
  o += (size_t)kRec * N;
  if (c->energy) {
    HIPCHK(c, hipMemcpy(c->T[q_last], o, sizeof(double) * N, hipMemcpyHostToDevice));
    o += N;
  }
  if (c->has_mech) {
    HIPCHK(c, hipMemcpy(c->theta, o, sizeof(double) * c->K * N, hipMemcpyHostToDevice));
    o += (size_t)c->K * N;
  }
  if (c->electrode) {
    double *dst[] = {c->pel, c->iv, c->ia, c->ped};
    for (double *d : dst) {
      HIPCHK(c, hipMemcpy(d, o, sizeof(double) * N, hipMemcpyHostToDevice));
      o += N;
    }
    HIPCHK(c, hipMemcpy(c->d_phi_line, o, sizeof(double) * c->n_lines, hipMemcpyHostToDevice));
  }
  return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err : "null context"; }

void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  drop_graph(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->timing) lbm_set_timing(c, 0);
  double *bufs[] = {c->pop[0], c->pop[1], c->phi, c->kfac, c->Tfield, c->X0, c->Plat, c->rA, c->rRT, c->rFk,
                    c->rrho, c->rY, c->rqd, c->rec[0], c->rec[1], c->T[0], c->T[1], c->srcsum, c->theta, c->rEs, c->faradaic, c->macro, c->partials,
                    c->iv, c->ia, c->pel, c->ped, c->omega_n, c->uel,
                    c->d_phi_line, c->d_target, c->d_p0, c->d_f0, c->d_p1,
                    c->iv_try, c->ia_try, c->pel_try, c->ped_try};
  for (double *b : bufs) dfree(b);
  dfree(c->colflag);
  dfree(c->d_line_off);
  dfree(c->theta_alt);
  dfree(c->win_sk);
  dfree(c->chem_tab);
  delete c;
}

}  // extern "C"
