// chem_jit.hip -- mechanism-specialised surface-chemistry kernel (Section 4).
//
// The local update is the same as k_chem's: backward Euler over n_sub
// sub-steps, n_newton Newton iterations per sub-step on the gas
// concentrations and all K coverages (eqs totalFluidReactionRate,
// molarToMassRates, surfaceMoleFractions, totalSurfaceReactionRate), then the
// extent-based conservative update and the species source (eq rho_pc).
//
// What differs is that the mechanism is fixed when lbm_set_mechanism is
// called, so its stoichiometry and Arrhenius constants are written into the
// kernel source as literals and the kernel is compiled for gfx950 with hiprtc.
// The generated code is straight-line and touches only the structurally
// non-zero entries:
//   - rates and their derivatives expand only the species a reaction names;
//   - the Jacobian G = sum_r nu_r (dq_r/dy)^T is assembled on its pattern;
//   - LU runs on the symbolic fill pattern in a fixed elimination order
//     without row exchanges, while every lane checks the partial-pivoting
//     condition |a_kk| >= |a_rk| on the partially eliminated column.  When
//     partial pivoting would have exchanged rows the lane redoes the Newton
//     step with a dense LU with partial pivoting, so the result is always
//     that of a partially pivoted solve.
// The elimination order comes from an analysis of Newton matrices sampled on
// the initial state (chem_choose_order): greedy minimum fill among the
// unknowns whose pivot dominates its partially eliminated column on every
// sample, which keeps the no-exchange path the common one.
// Rows are divided by the phase weight (phi for gas, Gamma for coverages), as
// in k_chem.  Kernels are cached per process by their source text.
#include "lbm_internal.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace {

struct Out {
  std::string s;
  void operator()(const char *fmt, ...) __attribute__((format(printf, 2, 3))) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s += buf;
    s += '\n';
  }
};

// Exact decimal-free literal of a double.
std::string lit(double v) {
  char b[64];
  std::snprintf(b, sizeof b, "%a", v);
  return std::string("(") + b + ")";
}

struct Gen {
  const ChemSpec &sp;
  int M, K, S, R;
  std::vector<std::vector<int>> st, nf, nb;
  std::vector<std::vector<bool>> in;   // species t appears in reaction r
  bool pat[16][16] = {};               // assembled pattern (with diagonal)
  bool lu[16][16] = {};                // pattern after fill
  std::vector<int> perm;               // elimination order

  explicit Gen(const ChemSpec &s) : sp(s) {
    M = sp.M;
    K = sp.K;
    S = M + K;
    R = sp.R;
    st.assign(R, std::vector<int>(S, 0));
    nf = nb = st;
    in.assign(R, std::vector<bool>(S, false));
    for (int r = 0; r < R; ++r)
      for (int t = 0; t < S; ++t) {
        nf[r][t] = sp.nu_f[r][t];
        nb[r][t] = sp.nu_b[r][t];
        st[r][t] = nb[r][t] - nf[r][t];
        in[r][t] = nf[r][t] != 0 || nb[r][t] != 0;
      }
    for (int s = 0; s < S; ++s) pat[s][s] = true;
    for (int r = 0; r < R; ++r)
      for (int s = 0; s < S; ++s)
        if (st[r][s])
          for (int t = 0; t < S; ++t)
            if (in[r][t]) pat[s][t] = true;
    for (int k = 0; k < S; ++k) perm.push_back(sp.perm[k]);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) lu[i][j] = pat[i][j];
    for (int k = 0; k < S; ++k) {
      const int pk = perm[k];
      for (int r = k + 1; r < S; ++r) {
        const int pr = perm[r];
        if (!lu[pr][pk]) continue;
        for (int c = k + 1; c < S; ++c)
          if (lu[pk][perm[c]]) lu[pr][perm[c]] = true;
      }
    }
  }

  bool active(int r, int dirn) const {   // forward (0) / backward (1) branch present
    return dirn == 0 ? sp.A_f[r] != 0.0 : sp.A_b[r] != 0.0;
  }

  // k * prod_t C_t^nu_t, optionally differentiated with respect to C_w.
  std::string product(int r, int dirn, int w) const {
    const std::vector<int> &nu = dirn == 0 ? nf[r] : nb[r];
    std::string e = dirn == 0 ? "kf" : "kb";
    for (int t = 0; t < S; ++t) {
      int p = nu[t];
      if (t == w) {
        if (p == 0) return "";
        if (p > 1) e += " * " + std::to_string(p) + ".0";
        p -= 1;
      }
      for (int i = 0; i < p; ++i) e += " * C[" + std::to_string(t) + "]";
    }
    return e;
  }

  std::string rate(int r) const {
    std::string f = active(r, 0) ? product(r, 0, -1) : "";
    std::string b = active(r, 1) ? product(r, 1, -1) : "";
    if (f.empty() && b.empty()) return "0.0";
    if (b.empty()) return f;
    if (f.empty()) return "-(" + b + ")";
    return "(" + f + ") - (" + b + ")";
  }

  std::string drate(int r, int w) const {
    std::string f = active(r, 0) ? product(r, 0, w) : "";
    std::string b = active(r, 1) ? product(r, 1, w) : "";
    if (f.empty() && b.empty()) return "";
    if (b.empty()) return f;
    if (f.empty()) return "-(" + b + ")";
    return "(" + f + ") - (" + b + ")";
  }

  // Weight of reaction r in the balance of species s, relative to the row
  // coefficient (h / phi for gas rows, h / Gamma_s for coverage rows):
  // gas rows take a^(s) of the reaction's surface (phi for a homogeneous
  // reaction), coverage rows 1 (l_TPB / a^(s)_s for a TPB edge reaction).
  std::string weight(int r, int s) const {
    if (s < M) return sp.kind[r] == 1 ? std::string("phi") : lit(sp.w_r[r]);
    if (sp.kind[r] == 2) return lit(sp.l_tpb / sp.a_k[s - M]);
    return "";
  }

  // "x" scaled by c * weight(r, s) as an accumulation statement tail.
  std::string acc(int r, int s, int c, const std::string &x) const {
    std::string w = weight(r, s);
    std::string e = w.empty() ? x : w + " * " + x;
    if (c == 1) return " += " + e;
    if (c == -1) return " -= " + e;
    return " += " + std::to_string(c) + ".0 * " + e;
  }

  static std::string times(int c, const char *x) {
    if (c == 1) return std::string(" += ") + x;
    if (c == -1) return std::string(" -= ") + x;
    return std::string(" += ") + std::to_string(c) + ".0 * " + x;
  }

  void concentrations(Out &o) const {
    for (int a = 0; a < M; ++a) o("      C[%d] = y[%d];", a, a);
    for (int s = M; s < S; ++s) o("      C[%d] = %s * y[%d];", s, lit(sp.gam_k[s - M]).c_str(), s);
  }

  // J <- I - coef_s G, b <- -(y - y0) + coef_s P at the iterate y.
  void assemble(Out &o) const {
    concentrations(o);
    for (int s = 0; s < S; ++s) {
      o("      P[%d] = 0.0;", s);
      for (int t = 0; t < S; ++t)
        if (pat[s][t]) o("      J[%d][%d] = 0.0;", s, t);
    }
    for (int r = 0; r < R; ++r) {
      if (!active(r, 0) && !active(r, 1)) continue;
      o("      {  // reaction %d", r);
      o("        const double kf = sk[%d][lane], kb = sk[%d][lane];", 2 * r, 2 * r + 1);
      o("        (void)kf; (void)kb;");
      o("        const double q = %s;", rate(r).c_str());
      for (int s = 0; s < S; ++s)
        if (st[r][s]) o("        P[%d]%s;", s, acc(r, s, st[r][s], "q").c_str());
      for (int t = 0; t < S; ++t) {
        if (!in[r][t]) continue;
        const std::string d = drate(r, t);
        if (d.empty()) continue;
        if (t < M)
          o("        { const double d = %s;", d.c_str());
        else
          o("        { const double d = %s * (%s);", lit(sp.gam_k[t - M]).c_str(), d.c_str());
        for (int s = 0; s < S; ++s)
          if (st[r][s]) o("          J[%d][%d]%s;", s, t, acc(r, s, st[r][s], "d").c_str());
        o("        }");
      }
      o("      }");
    }
    for (int s = 0; s < S; ++s) {
      const std::string cfs = s < M ? std::string("cg") : "cs" + std::to_string(s);
      const char *cf = cfs.c_str();
      for (int t = 0; t < S; ++t) {
        if (!pat[s][t]) continue;
        if (s == t)
          o("      J[%d][%d] = 1.0 - %s * J[%d][%d];", s, t, cf, s, t);
        else
          o("      J[%d][%d] = -%s * J[%d][%d];", s, t, cf, s, t);
      }
      o("      b[%d] = -(y[%d] - y0(%d)) + %s * P[%d];", s, s, s, cf, s);
    }
  }

  // Sparse LU without exchanges, forward substitution fused, then back
  // substitution; `bad` records where partial pivoting would exchange rows.
  void factor_solve(Out &o) const {
    bool init[16][16];
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) init[i][j] = pat[i][j];
    for (int k = 0; k < S; ++k) {
      const int pk = perm[k];
      o("      {  // pivot %d (species %d)", k, pk);
      o("        const double d = J[%d][%d], ad = fabs(d);", pk, pk);
      for (int r = k + 1; r < S; ++r)
        if (lu[perm[r]][pk]) o("        bad |= fabs(J[%d][%d]) > ad;", perm[r], pk);
      o("        const double inv = 1.0 / d;");
      o("        J[%d][%d] = inv;", pk, pk);
      for (int r = k + 1; r < S; ++r) {
        const int pr = perm[r];
        if (!lu[pr][pk]) continue;
        o("        { const double l = J[%d][%d] * inv;", pr, pk);
        for (int c = k + 1; c < S; ++c) {
          const int pc = perm[c];
          if (!lu[pk][pc]) continue;
          if (init[pr][pc]) {
            o("          J[%d][%d] -= l * J[%d][%d];", pr, pc, pk, pc);
          } else {
            o("          J[%d][%d] = -l * J[%d][%d];", pr, pc, pk, pc);
            init[pr][pc] = true;
          }
        }
        o("          b[%d] -= l * b[%d]; }", pr, pk);
      }
      o("      }");
    }
    for (int k = S - 1; k >= 0; --k) {
      const int pk = perm[k];
      std::string e = "b[" + std::to_string(pk) + "]";
      for (int c = k + 1; c < S; ++c)
        if (lu[pk][perm[c]])
          e += " - J[" + std::to_string(pk) + "][" + std::to_string(perm[c]) + "] * b[" +
               std::to_string(perm[c]) + "]";
      o("      b[%d] = (%s) * J[%d][%d];", pk, e.c_str(), pk, pk);
    }
  }

  // Dense LU with partial pivoting (first maximum on ties) on a private copy.
  void dense_solve(Out &o) const {
    o("      double A[%d][%d];", S, S + 1);
    o("#pragma unroll 1");
    o("      for (int i = 0; i < %d; ++i)", S);
    o("#pragma unroll 1");
    o("        for (int j = 0; j <= %d; ++j) A[i][j] = 0.0;", S);
    for (int s = 0; s < S; ++s) {
      for (int t = 0; t < S; ++t)
        if (pat[s][t]) o("      A[%d][%d] = J[%d][%d];", s, t, s, t);
      o("      A[%d][%d] = b[%d];", s, S, s);
    }
    o("#pragma unroll 1");
    o("      for (int k = 0; k < %d; ++k) {", S);
    o("        int p = k;");
    o("        double amax = fabs(A[k][k]);");
    o("#pragma unroll 1");
    o("        for (int r = k + 1; r < %d; ++r) {", S);
    o("          const double v = fabs(A[r][k]);");
    o("          if (v > amax) { amax = v; p = r; }");
    o("        }");
    o("        if (p != k) {");
    o("#pragma unroll 1");
    o("          for (int c = k; c <= %d; ++c) { const double t = A[k][c]; A[k][c] = A[p][c]; A[p][c] = t; }", S);
    o("        }");
    o("        const double inv = 1.0 / A[k][k];");
    o("#pragma unroll 1");
    o("        for (int r = k + 1; r < %d; ++r) {", S);
    o("          const double l = A[r][k] * inv;");
    o("#pragma unroll 1");
    o("          for (int c = k + 1; c <= %d; ++c) A[r][c] -= l * A[k][c];", S);
    o("        }");
    o("      }");
    o("#pragma unroll 1");
    o("      for (int k = %d; k >= 0; --k) {", S - 1);
    o("        double x = A[k][%d];", S);
    o("#pragma unroll 1");
    o("        for (int c = k + 1; c < %d; ++c) x -= A[k][c] * A[c][%d];", S, S);
    o("        A[k][%d] = x / A[k][k];", S);
    o("      }");
    for (int s = 0; s < S; ++s) o("      b[%d] = A[%d][%d];", s, s, S);
  }

  std::string source() const {
    Out o;
    int nnz_pat = 0, nnz_lu = 0;
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) {
        nnz_pat += pat[i][j];
        nnz_lu += lu[i][j];
      }
    std::string order;
    for (int k = 0; k < S; ++k) order += " " + std::to_string(perm[k]);
    o("// Generated surface-chemistry kernel: M=%d gas species, K=%d surface species, R=%d reactions.", M,
      K, R);
    o("// Newton matrix pattern %d of %d entries, %d after fill; elimination order:%s", nnz_pat, S * S, nnz_lu,
      order.c_str());
    o("#define KREC %d", kRec);
    o("#define KRECSRC %d", kRecSrc);
    o("extern \"C\" __global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))\n    lbm_chem_specialized(");
    o("    const int N, const double *__restrict__ Tn, const double *__restrict__ phin,");
    o("    const double *__restrict__ rrho, double *__restrict__ theta, double *__restrict__ rec,");
    o("    double *__restrict__ srcsum, const double *__restrict__ faradaic, const int fuel,");
    o("    const int product, const double dt, const double rho_unit, const double gam,");
    o("    const double a_s, const double *__restrict__ ped, const double *__restrict__ pel,");
    o("    double *__restrict__ ivo, const double *__restrict__ omega, double *__restrict__ uel,");
    o("    const int dry, const double F_C, const double a_el, const double dx, const double inv_e_unit) {");
    o("  __shared__ double sk[%d][64];   // rate constants of this lane's node", 2 * R);
    o("  __shared__ double sy[%d][64];   // state at the start of the sub-step", S);
    o("  const int lane = threadIdx.x;");
    o("  const int n = blockIdx.x * 64 + lane;");
    o("  if (n >= N) return;");
    o("  const double T = Tn[n], phi = phin[n];");
    o("  const double inv_RT = 1.0 / (%s * T);", lit(sp.R_U).c_str());
    for (int r = 0; r < R; ++r)
      for (int dirn = 0; dirn < 2; ++dirn) {
        const double A = dirn == 0 ? sp.A_f[r] : sp.A_b[r];
        const double Ea = dirn == 0 ? sp.Ea_f[r] : sp.Ea_b[r];
        if (A == 0.0)
          o("  sk[%d][lane] = 0.0;", 2 * r + dirn);
        else if (Ea == 0.0)
          o("  sk[%d][lane] = %s;", 2 * r + dirn, lit(A).c_str());
        else
          o("  sk[%d][lane] = %s * exp(-%s * inv_RT);", 2 * r + dirn, lit(A).c_str(), lit(Ea).c_str());
      }
    // charge transfer: Butler-Volmer factors at dPhi = Phi_electrode - Phi_electrolyte
    o("  const double fpot = pel ? F_C * (ped[n] - pel[n]) * inv_RT : 0.0;");
    o("  (void)fpot; (void)omega; (void)a_el; (void)dx; (void)inv_e_unit;");
    for (int r = 0; r < R; ++r)
      if (sp.charge_z[r]) {
        const double z = (double)sp.charge_z[r];
        o("  sk[%d][lane] *= exp(%s * fpot);", 2 * r, lit(sp.beta_ct[r] * z).c_str());
        o("  sk[%d][lane] *= exp(%s * fpot);", 2 * r + 1, lit(-(1.0 - sp.beta_ct[r]) * z).c_str());
      }
    o("  double iv = 0.0;   // charge released per unit volume over the step / dt");
    o("#define y0(s) sy[s][lane]");
    o("  double src[%d];", M);
    for (int a = 0; a < M; ++a) {
      o("  y0(%d) = rrho[(size_t)%d * N + n] * rho_unit / %s;", a, a, lit(sp.m[a]).c_str());
      o("  src[%d] = 0.0;", a);
    }
    for (int k = 0; k < K; ++k) o("  y0(%d) = theta[(size_t)%d * N + n];", M + k, k);
    o("  const double h = dt / %d.0;", sp.n_sub);
    o("  const double cg = h / phi;   // gas rows (phi c); coverage rows (Gamma theta):");
    for (int s = M; s < S; ++s) o("  const double cs%d = h / %s;", s, lit(sp.gam_k[s - M]).c_str());
    o("  (void)gam; (void)a_s;");
    o("#pragma unroll 1");
    o("  for (int sub = 0; sub < %d; ++sub) {", sp.n_sub);
    o("    double y[%d];", S);
    for (int s = 0; s < S; ++s) o("    y[%d] = y0(%d);", s, s);
    o("#pragma unroll 1");
    o("    for (int it = 0; it < %d; ++it) {", sp.n_newton);
    o("      double C[%d], P[%d], J[%d][%d], b[%d];", S, S, S, S, S);
    o("      bool bad = false;");
    assemble(o);
    factor_solve(o);
    o("      if (bad) {  // partial pivoting would exchange rows: dense pivoted solve");
    assemble(o);
    dense_solve(o);
    o("      }");
    for (int s = 0; s < S; ++s) o("      y[%d] += b[%d];", s, s);
    o("    }");
    o("    // extents at the implicit state; conservative update of both phases");
    o("    double C[%d], dn[%d];", S, S);
    concentrations(o);
    for (int s = 0; s < S; ++s) o("    dn[%d] = 0.0;", s);
    o("    double ze = 0.0;   // sum_r z_r xi_r");
    for (int r = 0; r < R; ++r) {
      if (!active(r, 0) && !active(r, 1)) continue;
      o("    {");
      o("      const double kf = sk[%d][lane], kb = sk[%d][lane];", 2 * r, 2 * r + 1);
      o("      (void)kf; (void)kb;");
      o("      const double dxi = h * (%s);", rate(r).c_str());
      for (int s = 0; s < S; ++s)
        if (st[r][s]) o("      dn[%d]%s;", s, acc(r, s, st[r][s], "dxi").c_str());
      if (sp.charge_z[r]) o("      ze += %d.0 * dxi;", sp.charge_z[r]);
      o("    }");
    }
    if (sp.has_ct) o("    iv += F_C * %s * ze / dt;   // eq volumetricCurrent", lit(sp.l_tpb).c_str());
    o("    (void)ze;");
    for (int k = 0; k < K; ++k) o("    y0(%d) += dn[%d] / %s;", M + k, M + k, lit(sp.gam_k[k]).c_str());
    for (int a = 0; a < M; ++a) {
      o("    { const double dgas = dn[%d];   // mol per m^3 of REV", a);
      o("      y0(%d) += dgas / phi;", a);
      o("      src[%d] += dgas * %s / rho_unit; }", a, lit(sp.m[a]).c_str());
    }
    o("  }");
    o("  if (ivo) ivo[n] = iv;");
    o("  if (dry) return;   // a trial of the current control: only the current is wanted");
    o("  if (uel) {         // electrical work out, ohmic heat in");
    o("    const double p_elec = fabs(ped[n] - pel[n]) * iv;");
    o("    const double p_om = (a_el / %s) * iv * iv * omega[n] * dx;", lit(sp.l_tpb > 0 ? sp.l_tpb : 1.0).c_str());
    o("    uel[n] = (p_om - p_elec) * dt * inv_e_unit;");
    o("  }");
    o("  if (faradaic) {");
    o("    const double r = faradaic[n] * dt;");
    for (int a = 0; a < M; ++a) {
      o("    if (fuel == %d) src[%d] -= r * %s / rho_unit;", a, a, lit(sp.m[a]).c_str());
      o("    if (product == %d) src[%d] += r * %s / rho_unit;", a, a, lit(sp.m[a]).c_str());
    }
    o("  }");
    o("  double ssum = 0.0;");
    for (int a = 0; a < M; ++a) {
      o("  rec[(size_t)(KRECSRC + %d) * N + n] = src[%d];", a, a);
      o("  ssum += src[%d];", a);
    }
    o("  srcsum[n] = ssum;");
    for (int k = 0; k < K; ++k) o("  theta[(size_t)%d * N + n] = y0(%d);", k, M + k);
    o("}");
    return o.s;
  }
};

struct Compiled {
  hipModule_t mod;
  hipFunction_t fn;
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, Compiled> g_cache;

}  // namespace

std::string chem_specialized_source(const ChemSpec &spec) { return Gen(spec).source(); }

void chem_choose_order(ChemSpec &sp, int ns, const double *T, const double *phi, const double *C, double h,
                       double a_s, double gam) {
  const int M = sp.M, S = sp.M + sp.K, R = sp.R;
  // Newton matrices J = I - coef_s sum_r st_rs dq_r/dy_t at the samples
  std::vector<double> J((size_t)ns * S * S, 0.0);
  bool pat[16][16] = {};
  for (int j = 0; j < ns; ++j) {
    double *A = &J[(size_t)j * S * S];
    const double *c = C + (size_t)j * S;
    const double inv_RT = 1.0 / (sp.R_U * T[j]);
    for (int r = 0; r < R; ++r) {
      const double kf = sp.A_f[r] * std::exp(-sp.Ea_f[r] * inv_RT);
      const double kb = sp.A_b[r] * std::exp(-sp.Ea_b[r] * inv_RT);
      for (int t = 0; t < S; ++t) {
        if (!sp.nu_f[r][t] && !sp.nu_b[r][t]) continue;
        double df = sp.nu_f[r][t] ? kf * sp.nu_f[r][t] : 0.0;
        double db = sp.nu_b[r][t] ? kb * sp.nu_b[r][t] : 0.0;
        for (int u = 0; u < S; ++u) {
          const int ef = sp.nu_f[r][u] - (u == t ? 1 : 0), eb = sp.nu_b[r][u] - (u == t ? 1 : 0);
          for (int i = 0; i < ef; ++i) df *= c[u];
          for (int i = 0; i < eb; ++i) db *= c[u];
        }
        const double d = (df - db) * (t < M ? 1.0 : sp.gam_k[t - M]);
        for (int s = 0; s < S; ++s) {
          const int st = sp.nu_b[r][s] - sp.nu_f[r][s];
          if (!st) continue;
          const double coef = s < M ? (sp.kind[r] == 1 ? h : h * sp.w_r[r] / phi[j])
                                    : h / sp.gam_k[s - M] * (sp.kind[r] == 2 ? sp.l_tpb / sp.a_k[s - M] : 1.0);
          A[s * S + t] -= coef * st * d;
          pat[s][t] = true;
        }
      }
    }
    for (int s = 0; s < S; ++s) {
      A[s * S + s] += 1.0;
      pat[s][s] = true;
    }
  }
  std::vector<int> rem;
  for (int s = 0; s < S; ++s) rem.push_back(s);
  int nperm = 0;
  while (!rem.empty()) {
    int best = -1, best_fill = 0;
    double best_ratio = 0.0;
    for (int k : rem) {
      double ratio = 0.0;
      for (int j = 0; j < ns; ++j) {
        const double *A = &J[(size_t)j * S * S];
        const double d = std::fabs(A[k * S + k]);
        for (int r : rem)
          if (r != k) {
            const double v = std::fabs(A[r * S + k]);
            ratio = std::fmax(ratio, d > 0.0 ? v / d : (v > 0.0 ? INFINITY : 0.0));
          }
      }
      int fill = 0;
      for (int r : rem)
        if (r != k && pat[r][k])
          for (int c2 : rem)
            if (c2 != k && pat[k][c2] && !pat[r][c2]) ++fill;
      const bool ok = ratio <= 0.5, best_ok = best_ratio <= 0.5;
      bool take = best < 0;
      if (!take && ok != best_ok) take = ok;
      else if (!take && ok) take = fill < best_fill || (fill == best_fill && ratio < best_ratio);
      else if (!take) take = ratio < best_ratio;
      if (take) {
        best = k;
        best_fill = fill;
        best_ratio = ratio;
      }
    }
    // eliminate `best` on every sample and in the pattern
    for (int j = 0; j < ns; ++j) {
      double *A = &J[(size_t)j * S * S];
      const double d = A[best * S + best];
      for (int r : rem) {
        if (r == best || A[r * S + best] == 0.0) continue;
        const double l = A[r * S + best] / d;
        for (int c2 : rem)
          if (c2 != best) A[r * S + c2] -= l * A[best * S + c2];
      }
    }
    for (int r : rem)
      if (r != best && pat[r][best])
        for (int c2 : rem)
          if (c2 != best && pat[best][c2]) pat[r][c2] = true;
    sp.perm[nperm++] = best;
    rem.erase(std::find(rem.begin(), rem.end(), best));
  }
}

hipError_t chem_specialize(const ChemSpec &spec, hipFunction_t *fn, std::string *log) {
  const std::string src = chem_specialized_source(spec);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find({dev, src});
  if (it != g_cache.end()) {
    *fn = it->second.fn;
    return hipSuccess;
  }
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "lbm_chem_specialized.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS) {
    if (log) *log = "hiprtcCreateProgram failed";
    return hipErrorInvalidValue;
  }
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=fast",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (rc != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string l(n + 1, '\0');
    hiprtcGetProgramLog(prog, &l[0]);
    if (log) *log = "hiprtc: " + l;
    hiprtcDestroyProgram(&prog);
    return hipErrorInvalidValue;
  }
  size_t code_size = 0;
  hiprtcGetCodeSize(prog, &code_size);
  std::vector<char> code(code_size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  Compiled c;
  e = hipModuleLoadData(&c.mod, code.data());
  if (e != hipSuccess) return e;
  e = hipModuleGetFunction(&c.fn, c.mod, "lbm_chem_specialized");
  if (e != hipSuccess) return e;
  g_cache[{dev, src}] = c;
  *fn = c.fn;
  return hipSuccess;
}

hipError_t launch_chem_specialized(hipFunction_t fn, const ChemParams &cp, hipStream_t s) {
  int N = cp.N;
  const double *T = cp.T, *phi = cp.phi, *rrho = cp.rrho, *far = cp.faradaic;
  double *theta = cp.theta, *rec = cp.rec, *srcsum = cp.srcsum;
  int fuel = cp.fuel, product = cp.product;
  double dt = cp.dt, rho_unit = cp.rho_unit, gam = cp.gamma, a_s = cp.a_s;
  const double *ped = cp.ped, *pel = cp.pel, *omega = cp.omega;
  double *iv = cp.iv, *uel = cp.uel;
  int dry = cp.dry;
  double F_C = cp.F_C, a_el = cp.a_el, dx = cp.dx, inv_e_unit = cp.inv_e_unit;
  void *args[] = {&N, &T, &phi, &rrho, &theta, &rec, &srcsum, &far, &fuel, &product, &dt, &rho_unit, &gam, &a_s,
                  &ped, &pel, &iv, &omega, &uel, &dry, &F_C, &a_el, &dx, &inv_e_unit};
  const unsigned nb = (unsigned)((N + 63) / 64);
  return hipModuleLaunchKernel(fn, nb, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}
