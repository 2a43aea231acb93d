// lbm_adjoint.hip -- reverse (adjoint) of the isothermal, reaction-free step
// for the gradient of an outlet-flux objective with respect to the porosity
// field and the pore radius.
//
// Forward map of one step at one node (Sections 2-3): post-stream populations
// F_t (all lattices) -> moments -> composition, relaxation rates (eqs tauab,
// taua, betaa, tauak), species momenta (eq transform1 with the Knudsen terms),
// Knudsen force (eq netKnudsenForce), extended momentum equilibrium (eqs Pex,
// feqmix with the Galilean correction G from neighbour records) -> collision
// (eqs finalNumericalEquationsReactive, f) -> stream to F_{t+1}.
//
// The adjoint of one step runs in two passes over the nodes:
//   pass 1: lambda'_t = transpose of the stream applied to Lambda_{t+1} (a
//           gather over the same pull addresses), then dJ/dG at the node;
//   pass 2: the adjoint of the node's collision: the population-level formulas
//           (Psi products, the collision update) are differentiated by hand;
//           the small coefficient map from the moments, phi and the Knudsen
//           factor to the collision coefficients (composition, rates, the M x M
//           solve, omega, u^ex, P^ex, the record rA, the objective) by a
//           hand-written reverse sweep (coef_map_reverse) that reuses the
//           solve's factorisation for the transposed system.  Lambda_t =
//           explicit population terms + the moment chain; phi and the Knudsen
//           factor accumulate their adjoints.
// Objective: J = (1/T) sum_{t=1..T} sum_{x = nx-1} j_{s,x}(F_t) / m_s, the
// solved momentum of species s through the last x plane, averaged over the
// collision steps (time levels 0..T-1).
#include "lbm_device.h"

namespace {

// Value of a coefficient-map quantity (the map is written once for its scalar type).
__device__ __forceinline__ double val(double a) { return a; }

// ---- coefficient map --------------------------------------------------------
// Inputs: raw lattice sums s0_l = sum_i f_li, s1_ld = sum_i f_li c_id (species
// l < M, momentum l = M), the Galilean-correction gradient G (already x3),
// phi and the Knudsen factor kfac.  Everything the collision needs besides the
// populations themselves.
template <class S, int D, int M>
struct Coef {
  S beta[M], Y[M], iab[M][M], itk[M], pra[M], xs[M][D], v[D];
  S omega, gfac, xi[D], Pex[D], phirho, rA[D], N;
};

template <class S, int D, int M>
__device__ __forceinline__ void coef_map(const KParams &p, const S (&s0)[M + 1], const S (&s1)[M + 1][D],
                                         const S (&G)[D], S phi, S kfac, double T, int out_species,
                                         Coef<S, D, M> &c) {
  S rho_a[M], rs = s0[0] / phi;
  rho_a[0] = rs;
#pragma unroll
  for (int a = 1; a < M; ++a) {
    rho_a[a] = s0[a] / phi;
    rs = rs + rho_a[a];
  }
  S im{};
#pragma unroll
  for (int a = 0; a < M; ++a) {
    c.Y[a] = rho_a[a] / rs;
    im = im + c.Y[a] * p.inv_m[a];
  }
  double RaT[M];
#pragma unroll
  for (int a = 0; a < M; ++a) RaT[a] = p.theta_ref * p.mmin_over_m[a] * (T * p.inv_T_ref);
  S RT = c.Y[0] * RaT[0], Ps = rho_a[0] * RaT[0];
#pragma unroll
  for (int a = 1; a < M; ++a) {
    RT = RT + c.Y[a] * RaT[a];
    Ps = Ps + rho_a[a] * RaT[a];
  }
  const double Tr = T * p.inv_T_ref;
  const S dfac = (Tr * ::sqrt(Tr)) / Ps;             // D_ab(T, P) = D_ab^ref (T/T_ref)^1.5 / P
  S A[M][M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    S it = S{};
#pragma unroll
    for (int b = 0; b < M; ++b) {
      c.iab[a][b] = S{};
      if (b != a) {
        c.iab[a][b] = RaT[a] / (p.Dref[a * LBM_MMAX + b] * dfac * (im / p.inv_m[b]));   // eq tauab
        it = it + c.Y[b] * c.iab[a][b];
      }
    }
    c.beta[a] = it / (2.0 + it);                     // eq betaa
    c.itk[a] = p.knudsen ? RaT[a] / (kfac * ::sqrt(RaT[a])) : S{};   // eq tauak
#pragma unroll
    for (int b = 0; b < M; ++b) A[a][b] = (b == a) ? 1.0 + 0.5 * it + 0.5 * c.itk[a] : -0.5 * c.Y[a] * c.iab[a][b];
  }
  // second-order species momenta: A x = s1 (Gaussian elimination, no exchanges)
  S x[M][D];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) x[a][d] = s1[a][d];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const S inv = 1.0 / A[k][k];
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const S l = A[r][k] * inv;
#pragma unroll
      for (int cc = k + 1; cc < M; ++cc) A[r][cc] = A[r][cc] - l * A[k][cc];
#pragma unroll
      for (int d = 0; d < D; ++d) x[r][d] = x[r][d] - l * x[k][d];
    }
  }
#pragma unroll
  for (int k = M - 1; k >= 0; --k) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      S sacc = x[k][d];
#pragma unroll
      for (int cc = k + 1; cc < M; ++cc) sacc = sacc - A[k][cc] * x[cc][d];
      x[k][d] = sacc / A[k][k];
    }
  }
#pragma unroll
  for (int a = 0; a < M; ++a) {
    c.pra[a] = s0[a];
    const bool pos = val(s0[a]) > 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) c.xs[a][d] = pos ? x[a][d] / s0[a] : S{};
  }
  c.N = S{};
#pragma unroll
  for (int a = 0; a < M; ++a)
    if (a == out_species) c.N = x[a][0];
  // momentum lattice
  const S rho = s0[M] / phi;
  S u[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[d] = s1[M][d] / rho;
    c.v[d] = u[d] / phi;
  }
  c.omega = 1.0 / (p.nu / RT + 0.5);
  c.gfac = (2.0 - c.omega) / (2.0 * phi * rho * c.omega);
  c.phirho = phi * rho;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    S Fk = S{};
#pragma unroll
    for (int a = 0; a < M; ++a) Fk = Fk - x[a][d] * c.itk[a];      // eq netKnudsenForce
    c.Pex[d] = RT + c.v[d] * c.v[d] + c.gfac * G[d];
    c.xi[d] = (u[d] + Fk / (c.omega * rho)) / phi;                 // u^ex / phi
    c.rA[d] = rho * u[d] * (1.0 - 3.0 * RT) - rho * u[d] * u[d] * u[d] / (phi * phi);
  }
}

// Reverse of coef_map: given the adjoints cb of its outputs, the adjoints of
// s0, s1, phi and kfac (G is handled in pass 1).  Recomputes the forward
// values, then runs the chain rule backwards through every intermediate.
template <int D, int M>
__device__ __forceinline__ void coef_map_reverse(const KParams &p, const double (&s0)[M + 1],
                                                 const double (&s1)[M + 1][D], const double (&G)[D], double phi,
                                                 double kfac, double T, int out_species,
                                                 const Coef<double, D, M> &cb, double (&s0b)[M + 1],
                                                 double (&s1b)[M + 1][D], double &phib, double &kfacb) {
  // ---- forward values
  double rho_a[M], rs = 0.0, Y[M], im = 0.0, RaT[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    rho_a[a] = s0[a] / phi;
    rs += rho_a[a];
  }
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Y[a] = rho_a[a] / rs;
    im += Y[a] * p.inv_m[a];
    RaT[a] = p.theta_ref * p.mmin_over_m[a] * (T * p.inv_T_ref);
  }
  double RT = 0.0, Ps = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    RT += Y[a] * RaT[a];
    Ps += rho_a[a] * RaT[a];
  }
  const double Tr = T * p.inv_T_ref;
  const double dfac = Tr * ::sqrt(Tr) / Ps;
  double iab[M][M], it[M], beta[M], itk[M], A[M][M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    it[a] = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) {
      iab[a][b] = 0.0;
      if (b != a) {
        iab[a][b] = RaT[a] / (p.Dref[a * LBM_MMAX + b] * dfac * (im / p.inv_m[b]));
        it[a] += Y[b] * iab[a][b];
      }
    }
    beta[a] = it[a] / (2.0 + it[a]);
    itk[a] = p.knudsen ? RaT[a] / (kfac * ::sqrt(RaT[a])) : 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) A[a][b] = (b == a) ? 1.0 + 0.5 * it[a] + 0.5 * itk[a] : -0.5 * Y[a] * iab[a][b];
  }
  double LU[M][M], x[M][D];
#pragma unroll
  for (int a = 0; a < M; ++a) {
#pragma unroll
    for (int b = 0; b < M; ++b) LU[a][b] = A[a][b];
#pragma unroll
    for (int d = 0; d < D; ++d) x[a][d] = s1[a][d];
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double inv = 1.0 / LU[k][k];
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const double l = LU[r][k] * inv;
      LU[r][k] = l;                                  // multiplier kept for the transposed solve
#pragma unroll
      for (int cc = k + 1; cc < M; ++cc) LU[r][cc] -= l * LU[k][cc];
#pragma unroll
      for (int d = 0; d < D; ++d) x[r][d] -= l * x[k][d];
    }
  }
#pragma unroll
  for (int k = M - 1; k >= 0; --k)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double sacc = x[k][d];
#pragma unroll
      for (int cc = k + 1; cc < M; ++cc) sacc -= LU[k][cc] * x[cc][d];
      x[k][d] = sacc / LU[k][k];
    }
  const double rho = s0[M] / phi;
  double u[D], v[D], Fk[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[d] = s1[M][d] / rho;
    v[d] = u[d] / phi;
    Fk[d] = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) Fk[d] -= x[a][d] * itk[a];
  }
  const double omega = 1.0 / (p.nu / RT + 0.5);
  const double gfac = (2.0 - omega) / (2.0 * phi * rho * omega);

  // ---- reverse
  double rhob = 0.0, RTb = 0.0, omegab = cb.omega, gfacb = cb.gfac, ub[D], vb[D], Fkb[D], xb[M][D];
  phib = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ub[d] = 0.0;
    vb[d] = cb.v[d];
    Fkb[d] = 0.0;
  }
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) xb[a][d] = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    // rA_d = rho u_d (1 - 3RT) - rho u_d^3 / phi^2
    const double rAb = cb.rA[d], u3 = u[d] * u[d] * u[d];
    rhob += rAb * (u[d] * (1.0 - 3.0 * RT) - u3 / (phi * phi));
    ub[d] += rAb * (rho * (1.0 - 3.0 * RT) - 3.0 * rho * u[d] * u[d] / (phi * phi));
    RTb += rAb * (-3.0 * rho * u[d]);
    phib += rAb * (2.0 * rho * u3 / (phi * phi * phi));
    // xi_d = (u_d + Fk_d / (omega rho)) / phi
    const double xib = cb.xi[d];
    const double xi = (u[d] + Fk[d] / (omega * rho)) / phi;
    ub[d] += xib / phi;
    Fkb[d] += xib / (phi * omega * rho);
    omegab -= xib * Fk[d] / (phi * omega * omega * rho);
    rhob -= xib * Fk[d] / (phi * omega * rho * rho);
    phib -= xib * xi / phi;
    // Pex_d = RT + v_d^2 + gfac G_d
    RTb += cb.Pex[d];
    vb[d] += 2.0 * v[d] * cb.Pex[d];
    gfacb += cb.Pex[d] * G[d];
  }
  double itkb[M], itb[M], Yb[M], iabb[M][M], s0sp[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    itkb[a] = cb.itk[a];
    itb[a] = 0.0;
    Yb[a] = cb.Y[a];
    s0sp[a] = cb.pra[a];
#pragma unroll
    for (int b = 0; b < M; ++b) iabb[a][b] = cb.iab[a][b];
  }
  // Fk_d = - sum_a x_ad itk_a
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int a = 0; a < M; ++a) {
      xb[a][d] -= Fkb[d] * itk[a];
      itkb[a] -= Fkb[d] * x[a][d];
    }
  // phirho = phi rho
  phib += cb.phirho * rho;
  rhob += cb.phirho * phi;
  // gfac = (2 - omega) / (2 phi rho omega)
  omegab += gfacb * (-1.0 / (phi * rho * omega * omega));
  phib += gfacb * (-gfac / phi);
  rhob += gfacb * (-gfac / rho);
  // omega = 1 / (nu / RT + 1/2)
  RTb += omegab * omega * omega * p.nu / (RT * RT);
  // v = u / phi, u = s1_M / rho, rho = s0_M / phi
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ub[d] += vb[d] / phi;
    phib -= vb[d] * v[d] / phi;
    s1b[M][d] = ub[d] / rho;
    rhob -= ub[d] * u[d] / rho;
  }
  s0b[M] = rhob / phi;
  phib -= rhob * rho / phi;
  // N = x[s][0]; xs_ad = x_ad / s0_a
#pragma unroll
  for (int a = 0; a < M; ++a) {
    if (a == out_species) xb[a][0] += cb.N;
    if (s0[a] > 0.0) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        xb[a][d] += cb.xs[a][d] / s0[a];
        s0sp[a] -= cb.xs[a][d] * x[a][d] / (s0[a] * s0[a]);
      }
    }
  }
  // x = A^-1 s1: z = A^-T xb, s1b += z, Ab = - z x^T
  double z[M][D];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) z[a][d] = xb[a][d];
  // A^T = U^T L^T: forward with U^T, back with L^T (unit diagonal)
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double sacc = z[k][d];
#pragma unroll
      for (int r = 0; r < k; ++r) sacc -= LU[r][k] * z[r][d];
      z[k][d] = sacc / LU[k][k];
    }
#pragma unroll
  for (int k = M - 1; k >= 0; --k)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double sacc = z[k][d];
#pragma unroll
      for (int r = k + 1; r < M; ++r) sacc -= LU[r][k] * z[r][d];
      z[k][d] = sacc;
    }
#pragma unroll
  for (int a = 0; a < M; ++a) {
#pragma unroll
    for (int d = 0; d < D; ++d) s1b[a][d] = z[a][d];
#pragma unroll
    for (int b = 0; b < M; ++b) {
      double Ab = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) Ab -= z[a][d] * x[b][d];
      if (b == a) {
        itb[a] += 0.5 * Ab;
        itkb[a] += 0.5 * Ab;
      } else {
        Yb[a] -= 0.5 * Ab * iab[a][b];
        iabb[a][b] -= 0.5 * Ab * Y[a];
      }
    }
  }
  kfacb = 0.0;
  double dfacb = 0.0, imb = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    if (p.knudsen) kfacb -= itkb[a] * itk[a] / kfac;          // itk = sqrt(R_a T) / kfac
    itb[a] += cb.beta[a] * 2.0 / ((2.0 + it[a]) * (2.0 + it[a]));
#pragma unroll
    for (int b = 0; b < M; ++b) {
      if (b == a) continue;
      Yb[b] += itb[a] * iab[a][b];
      iabb[a][b] += itb[a] * Y[b];
      dfacb -= iabb[a][b] * iab[a][b] / dfac;
      imb -= iabb[a][b] * iab[a][b] / im;
    }
  }
  const double Psb = -dfacb * dfac / Ps;
  double rhoab[M], rsb = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    rhoab[a] = Psb * RaT[a];
    Yb[a] += RTb * RaT[a] + imb * p.inv_m[a];
  }
#pragma unroll
  for (int a = 0; a < M; ++a) {
    rhoab[a] += Yb[a] / rs;
    rsb -= Yb[a] * Y[a] / rs;
  }
#pragma unroll
  for (int a = 0; a < M; ++a) {
    rhoab[a] += rsb;
    s0b[a] = s0sp[a] + rhoab[a] / phi;
    phib -= rhoab[a] * rho_a[a] / phi;
  }
}

// Psi_c(xi, P) and its partial derivatives.
__device__ __forceinline__ double dpsi_dxi(int c) { return c == 0 ? 0.0 : (c > 0 ? 0.5 : -0.5); }
__device__ __forceinline__ double dpsi_dP(int c) { return c == 0 ? -1.0 : 0.5; }
// Psi_c(v, v^2 + R) as a function of v
__device__ __forceinline__ double dpsiv_dv(int c, double v) { return c == 0 ? -2.0 * v : (c > 0 ? 0.5 + v : -0.5 + v); }

// Product over axes of Psi and its derivative along axis e.
template <int D>
__device__ __forceinline__ void psi_prod(int i, const double *xi, const double *P, double &prod,
                                         double *dxi, double *dP) {
  double f[D];
#pragma unroll
  for (int d = 0; d < D; ++d) f[d] = psi1(cdir(i, d), xi[d], P[d]);
  prod = 1.0;
#pragma unroll
  for (int d = 0; d < D; ++d) prod *= f[d];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    double o = 1.0;
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (d != e) o *= f[d];
    if (dxi) dxi[e] = dpsi_dxi(cdir(i, e)) * o;
    if (dP) dP[e] = dpsi_dP(cdir(i, e)) * o;
  }
}

// Psi_i(v, v^2 + R) and its derivative with respect to v_e.
template <int D>
__device__ __forceinline__ double psiv_prod(int i, const double *v, double R, double *dv) {
  double f[D];
#pragma unroll
  for (int d = 0; d < D; ++d) f[d] = psi1(cdir(i, d), v[d], v[d] * v[d] + R);
  double prod = 1.0;
#pragma unroll
  for (int d = 0; d < D; ++d) prod *= f[d];
  if (dv) {
#pragma unroll
    for (int e = 0; e < D; ++e) {
      double o = 1.0;
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (d != e) o *= f[d];
      dv[e] = dpsiv_dv(cdir(i, e), v[e]) * o;
    }
  }
  return prod;
}

// Node geometry from its index (grids only).
__device__ __forceinline__ Node node_of(const KParams &p, int n) {
  Node nd;
  nd.n = n;
  nd.x = n % p.nx;
  const int r = n / p.nx;
  nd.y = r % p.ny;
  nd.z = r / p.ny;
  nd.flag = (nd.x == 0 ? 1 : 0) | (nd.x == p.nx - 1 ? 2 : 0);
  return nd;
}

// Node at integer offset (dx, dy, dz) with periodic wrap in y, z and in x when x
// is periodic; -1 when it leaves a non-periodic x end.
__device__ __forceinline__ int offset_node(const KParams &p, const Node &nd, int dx, int dy, int dz) {
  int x = nd.x + dx, y = nd.y + dy, z = nd.z + dz;
  if (x < 0 || x >= p.nx) {
    if (p.bc_lo != BC_PERIODIC) return -1;
    x += (x < 0) ? p.nx : -p.nx;
  }
  y += (y < 0) ? p.ny : 0;
  y -= (y >= p.ny) ? p.ny : 0;
  z += (z < 0) ? p.nz : 0;
  z -= (z >= p.nz) ? p.nz : 0;
  return x + p.nx * (y + p.ny * z);
}

template <int D, int M>
struct AdjParams {
  KParams k;                 // pin = f'_{t-1}, rec_prev = v_{t-1}, rA = rA_t, first_step = (t == 1)
  const double *lam_next;    // Lambda_{t+1} [L][Q][N]; NULL at t = T
  double *lam_cur;           // Lambda_t
  double *lamp;              // lambda'_t (pass 1 writes, pass 2 reads)
  double *gbar;              // dJ/dG [D][N]
  double *phibar, *kfacbar;  // [N] accumulated
  double *jacc;              // [N] objective, outlet nodes
  double wN;                 // 1 / (T m_s)
  int out_species;
};

// A node away from non-periodic x ends (1 <= x <= nx - 2, or x periodic): its
// post-collision populations are read only by the regular pulls of its neighbours
// (walls, inlets and outflow copies act on nodes at x = 0 and x = nx - 1, and only
// on directions whose source lies outside), and the Galilean-correction stencil
// of each neighbour reaches it only through the regular offset.
__device__ __forceinline__ bool regular_node(const KParams &p, const Node &nd) {
  return p.bc_lo == BC_PERIODIC || (nd.x >= 1 && nd.x <= p.nx - 2);
}

// nbr[i] = node at offset sgn c_i of a regular node (periodic wrap in y and z, and
// in x when x is periodic).
template <int D>
__device__ __forceinline__ void neighbours(const KParams &p, const Node &nd, int sgn, int (&nbr)[LQ<D>::Q]) {
  int xs[3], ys[3], zs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = sgn * (k - 1);
    int x = nd.x + c, y = nd.y + (D > 1 ? c : 0), z = nd.z + (D > 2 ? c : 0);
    x += (x < 0) ? p.nx : 0;
    x -= (x >= p.nx) ? p.nx : 0;
    y += (y < 0) ? p.ny : 0;
    y -= (y >= p.ny) ? p.ny : 0;
    z += (z < 0) ? p.nz : 0;
    z -= (z >= p.nz) ? p.nz : 0;
    xs[k] = x;
    ys[k] = y;
    zs[k] = z;
  }
#pragma unroll
  for (int i = 0; i < LQ<D>::Q; ++i)
    nbr[i] = xs[cdir(i, 0) + 1] + p.nx * ((D > 1 ? ys[cdir(i, 1) + 1] : nd.y) + p.ny * (D > 2 ? zs[cdir(i, 2) + 1] : nd.z));
}

// lambda'_t(x, l, i): sum of Lambda_{t+1} over the (node, direction) pairs whose
// pull at step t+1 reads the post-collision population (x, l, i).
template <int D, int M>
__device__ __forceinline__ void stream_transpose(const AdjParams<D, M> &a, const Node &nd,
                                                 double (&lp)[M + 1][LQ<D>::Q]) {
  constexpr int Q = LQ<D>::Q;
  const KParams &p = a.k;
  const int N = p.N;
#pragma unroll
  for (int l = 0; l <= M; ++l)
#pragma unroll
    for (int i = 0; i < Q; ++i) lp[l][i] = 0.0;
  if (!a.lam_next) return;
  if (regular_node(p, nd)) {
    // the only reader of (x, l, i) is the regular pull of x + c_i at step t + 1
    int nbr[LQ<D>::Q];
    neighbours<D>(p, nd, 1, nbr);
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int l = 0; l <= M; ++l) lp[l][i] = a.lam_next[(size_t)(l * Q + i) * N + nbr[i]];
    return;
  }
  KParams pn = p;
  pn.first_step = 0;                                  // geometry of the pull at step t+1
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = cdir(i, 0), cy = D > 1 ? cdir(i, 1) : 0, cz = D > 2 ? cdir(i, 2) : 0;
    int cand[3], cdirn[3];
    cand[0] = offset_node(p, nd, cx, cy, cz);        // regular
    cdirn[0] = i;
    cand[1] = offset_node(p, nd, 0, cy, cz);         // outflow copy along the same x
    cdirn[1] = i;
    cand[2] = nd.n;                                  // bounce-back
    cdirn[2] = Q - 1 - i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int y = cand[k];
      if (y < 0) continue;
      bool dup = false;
      for (int k2 = 0; k2 < k; ++k2) dup |= (cand[k2] == y && cdirn[k2] == cdirn[k]);
      if (dup) continue;
      const Node ny = node_of(pn, y);
      const PullGeo<D> g = pull_geo<D>(pn, ny);
      int dir;
      const int src = pull_addr<D>(pn, ny, g, cdirn[k], dir);
      if (src != nd.n || dir != i || inlet_kind<D>(pn, ny, cdirn[k]) != 0) continue;
#pragma unroll
      for (int l = 0; l <= M; ++l) lp[l][i] += a.lam_next[(size_t)(l * Q + cdirn[k]) * N + y];
    }
  }
}

// Moments, G and the stored populations of node n at step t.
template <int D, int M>
__device__ __forceinline__ void node_inputs(const KParams &p, const Node &nd, double (&f)[M + 1][LQ<D>::Q],
                                            double (&s0)[M + 1], double (&s1)[M + 1][D], double (&G)[D],
                                            double &phi) {
  constexpr int Q = LQ<D>::Q;
  const int n = nd.n;
  phi = p.phi[n];
  const bool inlet_node = is_inlet_node(p, nd);
  double vb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) vb[d] = inlet_node ? p.rec_prev[(size_t)d * p.N + n] : 0.0;
  const PullGeo<D> geo = pull_geo<D>(p, nd);
#pragma unroll
  for (int l = 0; l <= M; ++l) {
    pull_lattice<D, M, false>(p, nd, geo, l, phi, vb, inlet_node, f[l]);
    s0[l] = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) s1[l][d] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s0[l] += f[l][i];
#pragma unroll
      for (int d = 0; d < D; ++d) s1[l][d] += cdir(i, d) * f[l][i];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) G[d] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (cnorm2<D>(i) == 0) continue;
    const int m = nb_node<D>(p, nd, i);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int c = cdir(i, d);
      if (c != 0) G[d] += wdir<D>(i) * c * p.rA[(size_t)d * p.N + m];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) G[d] *= 3.0;
}

// Where the pass-2 kernel's registers allow it (one wave per SIMD has up to 512), its
// loads are issued ahead of their use: every lattice of the pull at once and the next
// direction's lambda' during the current one; larger forms keep them in order.
template <int D, int M>
constexpr bool kAdjAhead = D == 1 || (D == 2 && M <= 3);

// Adjoint of the population-level collision at fixed coefficients: the
// coefficient adjoints cb.  Directions outermost, so only per-species values of
// one direction are live; lam(l, i) reads lambda'_t, dotf[l] = sum_i lambda'_li f_li.
template <int D, int M, class Lam>
__device__ __forceinline__ void collision_adjoint(const KParams &p, double T, const Lam &lam,
                                                  const double (&dotf)[M + 1], const Coef<double, D, M> &c,
                                                  Coef<double, D, M> &cb) {
  constexpr int Q = LQ<D>::Q;
  double RaT[M];
#pragma unroll
  for (int a = 0; a < M; ++a) RaT[a] = p.theta_ref * p.mmin_over_m[a] * (T * p.inv_T_ref);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    cb.beta[a] = -2.0 * dotf[a];                      // d f'/d beta has -2 f
    cb.Y[a] = cb.itk[a] = cb.pra[a] = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) cb.iab[a][b] = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) cb.xs[a][d] = 0.0;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) cb.v[d] = cb.xi[d] = cb.Pex[d] = cb.rA[d] = 0.0;
  cb.omega = -dotf[M];
  cb.gfac = cb.phirho = cb.N = 0.0;
  bool pos[M];
#pragma unroll
  for (int a = 0; a < M; ++a) pos[a] = c.pra[a] > 0.0;
  // with kAdjAhead, lambda'(., i + 1) is loaded while direction i is worked on (the
  // loop stays rolled; one wave per SIMD has no other wave to hide the load latency)
  double lnext[M + 1];
  if constexpr (kAdjAhead<D, M>) {
#pragma unroll
    for (int l = 0; l <= M; ++l) lnext[l] = lam(l, 0);
  }
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    double lcur[M + 1];
    if constexpr (kAdjAhead<D, M>) {
#pragma unroll
      for (int l = 0; l <= M; ++l) lcur[l] = lnext[l];
      if (i + 1 < Q) {
#pragma unroll
        for (int l = 0; l <= M; ++l) lnext[l] = lam(l, i + 1);
      }
    }
    auto li = [&](int l) {                        // lambda'(l, i)
      if constexpr (kAdjAhead<D, M>) return lcur[l];
      else return lam(l, i);
    };
    double E[M], S[M], K[M], dlt[M], dE[M][D], dS[M][D], dltb[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      double xs[D];
#pragma unroll
      for (int d = 0; d < D; ++d) xs[d] = c.xs[a][d];
      E[a] = psiv_prod<D>(i, c.v, RaT[a], dE[a]);
      S[a] = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) dS[a][d] = 0.0;
      if (pos[a]) S[a] = psiv_prod<D>(i, xs, RaT[a], dS[a]);
      K[a] = 1.0;
#pragma unroll
      for (int d = 0; d < D; ++d) K[a] *= psi1(cdir(i, d), 0.0, RaT[a]);
      dlt[a] = c.pra[a] * (E[a] - S[a]);
      dltb[a] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const double beta = c.beta[a], Ya = c.Y[a], itk = c.itk[a];
      const double feq = c.pra[a] * E[a], fst = pos[a] ? c.pra[a] * S[a] : 0.0, fk = c.pra[a] * K[a];
      double cross = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) cross += c.iab[a][b] * dlt[b];
      const double Fai = Ya * cross + itk * (fst - fk);
      const double l = li(a);
      cb.beta[a] += l * (2.0 * feq + Fai);
      const double Fb = (beta - 1.0) * l;
      cb.Y[a] += Fb * cross;
#pragma unroll
      for (int b = 0; b < M; ++b) {
        cb.iab[a][b] += Fb * Ya * dlt[b];
        dltb[b] += Fb * Ya * c.iab[a][b];
      }
      cb.itk[a] += Fb * (fst - fk);
      const double feqb = 2.0 * beta * l, fstb = Fb * itk, fkb = -Fb * itk;
      cb.pra[a] += feqb * E[a] + (pos[a] ? fstb * S[a] : 0.0) + fkb * K[a];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        cb.v[d] += feqb * c.pra[a] * dE[a][d];
        cb.xs[a][d] += fstb * c.pra[a] * dS[a][d];
      }
    }
    // the cross-term differences dlt_b = pra_b (E_b - S_b)
#pragma unroll
    for (int b = 0; b < M; ++b) {
      cb.pra[b] += dltb[b] * (E[b] - S[b]);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        cb.v[d] += dltb[b] * c.pra[b] * dE[b][d];
        cb.xs[b][d] -= dltb[b] * c.pra[b] * dS[b][d];
      }
    }
    // momentum lattice
    double X, dX[D], dP[D];
    psi_prod<D>(i, c.xi, c.Pex, X, dX, dP);
    const double l = li(M);
    cb.omega += l * c.phirho * X;
    const double fexb = c.omega * l;
    cb.phirho += fexb * X;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      cb.xi[d] += fexb * c.phirho * dX[d];
      cb.Pex[d] += fexb * c.phirho * dP[d];
    }
  }
}

// ---- pass 1: lambda'_t and dJ/dG ------------------------------------------
template <int D, int M>
__global__ __launch_bounds__(128) void k_adj_pass1(const AdjParams<D, M> a) {
  constexpr int Q = LQ<D>::Q;
  const KParams &p = a.k;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= p.N) return;
  const int N = p.N;
  const Node nd = node_of(p, n);
  double lp[M + 1][Q];
  stream_transpose<D, M>(a, nd, lp);
#pragma unroll
  for (int l = 0; l <= M; ++l)
#pragma unroll
    for (int i = 0; i < Q; ++i) a.lamp[(size_t)(l * Q + i) * N + n] = lp[l][i];
  double f[M + 1][Q], s0[M + 1], s1[M + 1][D], G[D], phi;
  node_inputs<D, M>(p, nd, f, s0, s1, G, phi);
  Coef<double, D, M> c;
  coef_map<double, D, M>(p, s0, s1, G, phi, p.kfac[n], p.Tfield[n], a.out_species, c);
  // dJ/dG_d = gfac * dJ/dPex_d, from the momentum lattice only
  double Gb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) Gb[d] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double X, dP[D];
    psi_prod<D>(i, c.xi, c.Pex, X, nullptr, dP);
    const double fexb = c.omega * lp[M][i];
#pragma unroll
    for (int d = 0; d < D; ++d) Gb[d] += fexb * c.phirho * dP[d];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) a.gbar[(size_t)d * N + n] = Gb[d] * c.gfac;
}

// ---- pass 2: Lambda_t, phi and Knudsen-factor adjoints, objective ----------
template <int D, int M>
__global__ __launch_bounds__(64) void k_adj_pass2(const AdjParams<D, M> a) {
  constexpr int Q = LQ<D>::Q;
  const KParams &p = a.k;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= p.N) return;
  const int N = p.N;
  const Node nd = node_of(p, n);
  const double *lamp = a.lamp;
  auto lam = [&](int l, int i) { return lamp[(size_t)(l * Q + i) * N + n]; };
  // pull, moments and sum_i lambda'_li f_li; the populations are not kept
  const double phi = p.phi[n];
  double s0[M + 1], s1[M + 1][D], dotf[M + 1], G[D];
  {
    const bool inlet_node = is_inlet_node(p, nd);
    double vbp[D];
#pragma unroll
    for (int d = 0; d < D; ++d) vbp[d] = inlet_node ? p.rec_prev[(size_t)d * p.N + n] : 0.0;
    const PullGeo<D> geo = pull_geo<D>(p, nd);
    if constexpr (kAdjAhead<D, M>) {               // every lattice's loads in flight at once
#pragma unroll
      for (int l = 0; l <= M; ++l) {
      double f[Q];
      pull_lattice<D, M, false>(p, nd, geo, l, phi, vbp, inlet_node, f);
      double t0 = 0.0, t1[D], df = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) t1[d] = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        t0 += f[i];
#pragma unroll
        for (int d = 0; d < D; ++d) t1[d] += cdir(i, d) * f[i];
        df += lam(l, i) * f[i];
      }
#pragma unroll
      for (int ll = 0; ll <= M; ++ll)               // select without indexing by the run-time l
        if (ll == l) {
          s0[ll] = t0;
          dotf[ll] = df;
#pragma unroll
          for (int d = 0; d < D; ++d) s1[ll][d] = t1[d];
        }
      }
    } else {                                        // one lattice at a time (registers)
#pragma unroll 1
      for (int l = 0; l <= M; ++l) {
      double f[Q];
      pull_lattice<D, M, false>(p, nd, geo, l, phi, vbp, inlet_node, f);
      double t0 = 0.0, t1[D], df = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) t1[d] = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        t0 += f[i];
#pragma unroll
        for (int d = 0; d < D; ++d) t1[d] += cdir(i, d) * f[i];
        df += lam(l, i) * f[i];
      }
#pragma unroll
      for (int ll = 0; ll <= M; ++ll)               // select without indexing by the run-time l
        if (ll == l) {
          s0[ll] = t0;
          dotf[ll] = df;
#pragma unroll
          for (int d = 0; d < D; ++d) s1[ll][d] = t1[d];
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) G[d] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cnorm2<D>(i) == 0) continue;
      const int m = nb_node<D>(p, nd, i);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int cc = cdir(i, d);
        if (cc != 0) G[d] += wdir<D>(i) * cc * p.rA[(size_t)d * N + m];
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) G[d] *= 3.0;
  }
  const double kfac = p.kfac[n], T = p.Tfield[n];
  Coef<double, D, M> c, cb;
  coef_map<double, D, M>(p, s0, s1, G, phi, kfac, T, a.out_species, c);
  collision_adjoint<D, M>(p, T, lam, dotf, c, cb);

  // rA_t(x) feeds G of the nodes whose stencil reaches x
  if (regular_node(p, nd)) {                          // only the node at -c_i, for every i
    int nbr[Q];
    neighbours<D>(p, nd, -1, nbr);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cnorm2<D>(i) == 0) continue;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int cc = cdir(i, d);
        if (cc != 0) cb.rA[d] += 3.0 * wdir<D>(i) * cc * a.gbar[(size_t)d * N + nbr[i]];
      }
    }
  } else {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (cnorm2<D>(i) == 0) continue;
    const int cx = cdir(i, 0), cy = D > 1 ? cdir(i, 1) : 0, cz = D > 2 ? cdir(i, 2) : 0;
    const int cand0 = offset_node(p, nd, -cx, -cy, -cz);
    int cands[2] = {cand0, (cand0 == n) ? -1 : n};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int xx = cands[k];
      if (xx < 0) continue;
      if (nb_node<D>(p, node_of(p, xx), i) != n) continue;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int cc = cdir(i, d);
        if (cc != 0) cb.rA[d] += 3.0 * wdir<D>(i) * cc * a.gbar[(size_t)d * N + xx];
      }
    }
  }
  }
  // the inlet equilibria of step t+1 use this node's v_t and phi
  double phib = 0.0;
  if (a.lam_next) {
    KParams pn = p;
    pn.first_step = 0;
    if (is_inlet_node(pn, nd)) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int kind = inlet_kind<D>(pn, nd, i);
        if (!kind) continue;
        const InletSel in = inlet_sel(p, kind, -1);
#pragma unroll
        for (int l = 0; l <= M; ++l) {
          const double L = a.lam_next[(size_t)(l * Q + i) * N + n];
          double R, rho;
          if (l < M) {
            const InletSel is = inlet_sel(p, kind, l);
            R = is.RaT;
            rho = is.rho_a;
          } else {
            R = in.RT;
            rho = in.rho;
          }
          double dv[D];
          const double pr = psiv_prod<D>(i, c.v, R, dv);
          phib += L * rho * pr;                      // F^in = phi rho Psi(v, v^2 + R)
#pragma unroll
          for (int d = 0; d < D; ++d) cb.v[d] += L * phi * rho * dv[d];
        }
      }
    }
  }
  // objective
  if (nd.flag & 2) {
    a.jacc[n] += c.N * a.wN;
    cb.N += a.wN;
  }
  // moment-space adjoints: reverse sweep through the coefficient map
  double s0b[M + 1], s1b[M + 1][D], phib_c, kfacb;
  coef_map_reverse<D, M>(p, s0, s1, G, phi, kfac, T, a.out_species, cb, s0b, s1b, phib_c, kfacb);
#pragma unroll
  for (int l = 0; l <= M; ++l) {
    double keep = 1.0 - c.omega;                      // explicit f term of the collision
#pragma unroll
    for (int aa = 0; aa < M; ++aa)
      if (aa == l) keep = 1.0 - 2.0 * c.beta[aa];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double s = lam(l, i) * keep + s0b[l];
#pragma unroll
      for (int d = 0; d < D; ++d) s += cdir(i, d) * s1b[l][d];
      a.lam_cur[(size_t)(l * Q + i) * N + n] = s;
    }
  }
  a.phibar[n] += phib_c + phib;
  a.kfacbar[n] += kfacb;
}

// Initial populations are phi times a phi-free equilibrium: dJ/dphi += Lambda_1 . F_1 / phi.
template <int D, int M>
__global__ __launch_bounds__(256) void k_adj_initial(const AdjParams<D, M> a) {
  constexpr int Q = LQ<D>::Q;
  const KParams &p = a.k;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= p.N) return;
  const int N = p.N;
  double s = 0.0;
  for (int l = 0; l <= M; ++l)
    for (int i = 0; i < Q; ++i)
      s += a.lam_next[(size_t)(l * Q + i) * N + n] * static_cast<const double *>(p.pin)[(size_t)(l * Q + i) * N + n];
  a.phibar[n] += s / p.phi[n];
}

template <int D, int M>
hipError_t adj_dispatch_m(const KParams &k, const AdjBuffers &b, int stage, hipStream_t s) {
  AdjParams<D, M> a;
  a.k = k;
  a.lam_next = b.lam_next;
  a.lam_cur = b.lam_cur;
  a.lamp = b.lamp;
  a.gbar = b.gbar;
  a.phibar = b.phibar;
  a.kfacbar = b.kfacbar;
  a.jacc = b.jacc;
  a.wN = b.wN;
  a.out_species = b.out_species;
  if (stage == 1)
    hipLaunchKernelGGL((k_adj_pass1<D, M>), dim3((k.N + 127) / 128), dim3(128), 0, s, a);
  else if (stage == 2)
    hipLaunchKernelGGL((k_adj_pass2<D, M>), dim3((k.N + 63) / 64), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_adj_initial<D, M>), dim3((k.N + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <int D>
hipError_t adj_dispatch_d(const KParams &k, const AdjBuffers &b, int stage, hipStream_t s) {
  switch (k.M) {
    case 2: return adj_dispatch_m<D, 2>(k, b, stage, s);
    case 3: return adj_dispatch_m<D, 3>(k, b, stage, s);
    case 4: return adj_dispatch_m<D, 4>(k, b, stage, s);
    case 5: return adj_dispatch_m<D, 5>(k, b, stage, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int dim, const KParams &k, const AdjBuffers &b, int stage, hipStream_t s) {
  switch (dim) {
    case 1: return adj_dispatch_d<1>(k, b, stage, s);
    case 2: return adj_dispatch_d<2>(k, b, stage, s);
    case 3: return adj_dispatch_d<3>(k, b, stage, s);
  }
  return hipErrorInvalidValue;
}
