// HIP kernels of the mean-field reactive porous-media lattice Boltzmann step (gfx950).
//
// One time step is two or three launches:
//   k_species  : pull-stream of every lattice, moments, composition, relaxation
//                rates, the M x M species-momentum solve, the species collision
//                (Section 2.3, eq finalNumericalEquationsReactive) and the small
//                per-node records the next kernels need;
//   k_chem     : the local surface-chemistry update (Section 4.2), only when a
//                mechanism or a Faradaic source is installed; it writes the
//                species source of the step into the node records;
//   k_mixture  : momentum (eqs f_source, feqmix, Pex) and energy (eqs g_source,
//                geq_i, gstar) collisions, which need gradients of node records.
// The reaction populations of a step (eq fsourceHetero) are added to the
// species populations when the next step pulls them (source_population), so
// no pass rewrites the stored populations.  Keeping the chemistry out of
// k_species keeps that kernel a bandwidth kernel.
//
// Populations are FP64 SoA [lattice][direction][node], one thread per node,
// node index x-fastest so every direction is a coalesced (shifted) stream.
// Population streams and per-step records are moved with non-temporal loads
// and stores, so the L2 keeps what is re-read: the neighbouring nodes' records.
#include "lbm_device.h"

namespace {

// ---------------------------------------------------------------------------
// Species front half: pull, moments, composition, coefficients, solve.
// Shared by the step kernel and the moments kernel.
// ---------------------------------------------------------------------------
template <int D, int M>
struct SpeciesState {
  static constexpr int Q = LQ<D>::Q;
  double f[M][Q];
  double rho_a[M], jt[M][D], ja[M][D];
  double rho, u[D], v[D];
  double Y[M], inv_mix, T, RaT[M], RT;
  double inv_tau_ab[M][M], beta[M], inv_tk[M];
  double Fk[D];
  double sumg;
};

template <int D, int M, bool ENERGY, typename PT>
__device__ __forceinline__ void species_front(const KParams &p, const Node &nd, double phi,
                                              SpeciesState<D, M> &S) {
  constexpr int Q = LQ<D>::Q;
  const int n = nd.n;
  // velocity of this node at the previous step (inlet equilibria)
  double vb[D];
  const bool inlet_node = is_inlet_node(p, nd);
#pragma unroll
  for (int d = 0; d < D; ++d) vb[d] = inlet_node ? p.rec_prev[(size_t)d * p.N + n] : 0.0;
  const PullGeo<D> geo = pull_geo<D>(p, nd);

  // ---- momentum lattice: sum f = phi rho (eq fdensity), sum f c = rho u
  double sf = 0.0, jf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) jf[d] = 0.0;
  {
    double fm[Q];
    pull_lattice<D, M, true, PT>(p, nd, geo, M, phi, vb, inlet_node, fm);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      sf += fm[i];
#pragma unroll
      for (int d = 0; d < D; ++d) jf[d] += cdir(i, d) * fm[i];
    }
  }
  S.rho = sf / phi;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    S.u[d] = jf[d] / S.rho;
    S.v[d] = S.u[d] / phi;
  }
  // ---- energy lattice zeroth moment (eq g0momTotalEnergy)
  S.sumg = 0.0;
  if (ENERGY) {
    double g[Q];
    pull_lattice<D, M, true, PT>(p, nd, geo, M + 1, phi, vb, inlet_node, g);
    double sg = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) sg += g[i];
    S.sumg = sg;
  }
  // ---- species lattices
#pragma unroll
  for (int a = 0; a < M; ++a) pull_lattice<D, M, true, PT>(p, nd, geo, a, phi, vb, inlet_node, S.f[a]);
  // ---- species moments (eqs density1, momentum1)
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double s0 = 0.0, s1[D];
#pragma unroll
    for (int d = 0; d < D; ++d) s1[d] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s0 += S.f[a][i];
#pragma unroll
      for (int d = 0; d < D; ++d) s1[d] += cdir(i, d) * S.f[a][i];
    }
    S.rho_a[a] = s0 / phi;
#pragma unroll
    for (int d = 0; d < D; ++d) S.jt[a][d] = s1[d];
  }
  // ---- composition (Section 2.1)
  double rs = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) rs += S.rho_a[a];
  double im = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    S.Y[a] = S.rho_a[a] / rs;
    im += S.Y[a] * p.inv_m[a];
  }
  S.inv_mix = im;
  // ---- temperature (eq temperature with E - v^2/2, constant heat capacities)
  if (ENERGY) {
    const double E = S.sumg / (phi * S.rho);
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) v2 += S.v[d] * S.v[d];
    double cvm = 0.0, u0m = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      cvm += S.Y[a] * p.cv[a];
      u0m += S.Y[a] * p.uf[a];
    }
    S.T = (E - 0.5 * v2 - u0m) / cvm;
  } else {
    S.T = p.Tfield[n];
  }
  double RT = 0.0, Ps = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    S.RaT[a] = p.theta_ref * p.mmin_over_m[a] * (S.T * p.inv_T_ref);
    RT += S.Y[a] * S.RaT[a];
    Ps += S.rho_a[a] * S.RaT[a];
  }
  S.RT = RT;
  // ---- relaxation rates (eqs tauab, taua, betaa, tauak with the dimensional
  //      readings tau_ab = D_ab m_a m_b / (m R_U T), tau^k_a = D^k_a m_a / (R_U T))
  const double Tr = S.T * p.inv_T_ref;
  const double dfac = Tr * sqrt(Tr) / Ps;        // D_ab(T, P) = D_ab^ref (T/T_ref)^1.5 / P
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double it = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) {
      if (b == a) {
        S.inv_tau_ab[a][b] = 0.0;
        continue;
      }
      // 1/tau_ab = R_a T m / (D_ab m_b)
      const double iab = S.RaT[a] / (p.Dref[a * LBM_MMAX + b] * dfac * (im / p.inv_m[b]));
      S.inv_tau_ab[a][b] = iab;
      it += S.Y[b] * iab;
    }
    S.beta[a] = it / (2.0 + it);                 // 1/(2 tau_a + 1)
    if (p.knudsen) {
      const double kf = p.kfac[n];
      S.inv_tk[a] = S.RaT[a] / (kf * sqrt(S.RaT[a]));
    } else {
      S.inv_tk[a] = 0.0;
    }
  }
  // ---- second-order species momenta: (1 + 1/2tau_a + 1/2tau^k_a) j_a
  //      - sum_{b != a} Y_a / (2 tau_ab) j_b = j~_a  (eq transform1 with the
  //      Knudsen terms); column diagonally dominant -> elimination without pivoting
  double A[M][M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double it = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) it += (b != a) ? S.Y[b] * S.inv_tau_ab[a][b] : 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b)
      A[a][b] = (a == b) ? (1.0 + 0.5 * it + 0.5 * S.inv_tk[a]) : (-0.5 * S.Y[a] * S.inv_tau_ab[a][b]);
  }
  double rhs[M][D];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) rhs[a][d] = S.jt[a][d];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const double l = A[r][k] * inv;
#pragma unroll
      for (int c = k + 1; c < M; ++c) A[r][c] -= l * A[k][c];
#pragma unroll
      for (int d = 0; d < D; ++d) rhs[r][d] -= l * rhs[k][d];
    }
  }
#pragma unroll
  for (int k = M - 1; k >= 0; --k) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double s = rhs[k][d];
#pragma unroll
      for (int c = k + 1; c < M; ++c) s -= A[k][c] * S.ja[c][d];
      S.ja[k][d] = s / A[k][k];
    }
  }
  // ---- Knudsen force on the mixture (eq netKnudsenForce): F^k = -sum_b j_b / tau^k_b
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double fk = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) fk -= S.ja[b][d] * S.inv_tk[b];
    S.Fk[d] = fk;
  }
}

// ---------------------------------------------------------------------------
// k_species: one tile = 64 nodes x (M species + momentum [+ energy]) waves; a
// block holds kSpeciesTiles tiles (two for D3Q27 with five species), each
// meeting at barriers of its own.  Wave w pulls lattice w for its 64 nodes (one
// coalesced stream per direction, plus the previous step's reaction
// populations) and keeps only those Q populations in registers.  Lattice
// moments meet in LDS.  Then every wave evaluates the cheap per-node state
// (composition, temperature, R_a T) itself, and species wave a its own row of
// relaxation rates (1/tau_ab, beta_a, 1/tau^k_a) and of the M x M
// species-momentum system, published in LDS.  The momentum wave solves that
// system and publishes the second-order species momenta; the species waves then
// publish their Delta table and collide their own lattice while the momentum
// wave writes the node records.
// ---------------------------------------------------------------------------
template <int D, int M, bool ENERGY>
struct SpeciesShared {
  static constexpr int L = M + 1 + (ENERGY ? 1 : 0);
  static constexpr int Q = LQ<D>::Q;
  double m0[L][64];             // zeroth moments: phi rho_a, phi rho, phi rho E
  double x[M][D][64];           // second-order species momenta, from the momentum wave
  // records of the previous step around the block's nodes (reaction populations):
  // row r of directions, field (source of species 0..M-1, T, v), node x0 - 1 + j
  static constexpr int R = Q / 3, F = M + 1 + D, W = 64 + 2;
  union {
    struct {
      double m1[M + 1][D][64];  // first moments of species and momentum lattices
      double A[M][M][64];       // species-momentum system, row a from species wave a
      double itk[M][64];        // 1 / tau^k_a
      double stage[R][F][W];    // before the moments only
    } s;
    double dlt[M][Q][64];       // phi rho_c (Psi_i(v) - Psi_i(xi_c)), after the solves
  } u;
};

// The tile's 64 nodes lie on one x row, inside the x walls, and all exist:
// then the pull sources of the three c_x of one (c_y, c_z) row of directions are
// that row's nodes x - 1 .. x + 1, and the tile can stage them once.
template <int D>
__device__ __forceinline__ bool row_block(const KParams &p, const Node &nd, const PullGeo<D> &g, bool valid) {
  if (p.colflag || p.first_step) return false;
  const unsigned long long all = __builtin_amdgcn_read_exec();
  const unsigned long long good = __builtin_amdgcn_uicmp((valid && !g.lo_wall && !g.hi_wall) ? 1u : 0u, 0u, 33);
  if (all != ~0ull || good != ~0ull) return false;
  const int x0 = __builtin_amdgcn_readlane(nd.x, 0), x63 = __builtin_amdgcn_readlane(nd.x, 63);
  return x63 - x0 == 63;
}


// Record field fi of the previous step: source of species fi (< M), T (= M),
// v_{fi - M - 1}; a select, no branch.
template <int M>
__device__ __forceinline__ const double *src_field(const KParams &p, int fi) {
  const int plane = fi < M ? kRecSrc + fi : fi - M - 1;
  const double *r = p.rec_prev + (size_t)plane * p.N;
  return fi == M ? p.T_prev : r;
}

// Offset nx (y_s + ny z_s) of row r = (c_y + 1) + 3 (c_z + 1) of directions:
// source y_s = y - c_y, z_s = z - c_z, periodic.
template <int D>
__device__ __forceinline__ int row_offset(const KParams &p, int y, int z, int r) {
  int ys = y, zs = z;
  if (D > 1) { ys -= r % 3 - 1; ys += (ys < 0) ? p.ny : 0; ys -= (ys >= p.ny) ? p.ny : 0; }
  if (D > 2) { zs -= r / 3 - 1; zs += (zs < 0) ? p.nz : 0; zs -= (zs >= p.nz) ? p.nz : 0; }
  return p.nx * (ys + p.ny * zs);
}

// Staged records of a row tile, spread over its L waves: wave w loads the
// (row r, field fi) pairs k = r F + fi with k = w mod L at its 64 nodes' x, and
// the fields fi with R F + fi = w mod L at the two wave-end sources of every
// row (lane 2r: x0 - 1, lane 2r + 1: x0 + 64, periodic in x).  All nodes of a
// row tile share y and z, so the row offsets are wave-uniform.  load_stage
// only issues the loads, so that they overlap the pull; store_stage writes them.
template <int D, int M, bool ENERGY>
struct Stage {
  using SS = SpeciesShared<D, M, ENERGY>;
  static constexpr int R = SS::R, F = SS::F, L = SS::L;
  static constexpr int NC = (R * F + L - 1) / L, NH = (F + L - 1) / L;
  double c[NC], h[NH];
};

template <int D, int M, bool ENERGY>
__device__ __forceinline__ void load_stage(const KParams &p, const Node &nd, int w, int lane,
                                           Stage<D, M, ENERGY> &st) {
  using S = Stage<D, M, ENERGY>;
  constexpr int R = S::R, F = S::F, L = S::L;
  const int y = __builtin_amdgcn_readfirstlane(nd.y), z = __builtin_amdgcn_readfirstlane(nd.z);
#pragma unroll
  for (int m = 0; m < S::NC; ++m) {
    const int k = min(w + m * L, R * F - 1);   // the clamped pair is loaded again, not stored
    st.c[m] = src_field<M>(p, k % F)[row_offset<D>(p, y, z, k / F) + nd.x];
  }
  const int x0 = __builtin_amdgcn_readfirstlane(nd.x);
  const int xe = (lane & 1) ? (x0 + 64 >= p.nx ? x0 + 64 - p.nx : x0 + 64) : (x0 == 0 ? p.nx - 1 : x0 - 1);
  const int hy = xe + row_offset<D>(p, y, z, min(lane >> 1, R - 1));
  const int f0 = ((w - (R * F) % L) % L + L) % L;
#pragma unroll
  for (int m = 0; m < S::NH; ++m) {
    const int fi = min(f0 + m * L, F - 1);
    st.h[m] = src_field<M>(p, fi)[hy];
  }
}

template <int D, int M, bool ENERGY>
__device__ __forceinline__ void store_stage(int w, int lane, const Stage<D, M, ENERGY> &st,
                                            SpeciesShared<D, M, ENERGY> &sh) {
  using S = Stage<D, M, ENERGY>;
  constexpr int R = S::R, F = S::F, L = S::L;
#pragma unroll
  for (int m = 0; m < S::NC; ++m) {
    const int k = w + m * L;
    if (k < R * F) sh.u.s.stage[k / F][k % F][lane + 1] = st.c[m];
  }
  const int f0 = ((w - (R * F) % L) % L + L) % L;
#pragma unroll
  for (int m = 0; m < S::NH; ++m) {
    const int fi = f0 + m * L;
    if (fi < F && lane < 2 * R) sh.u.s.stage[lane >> 1][fi][(lane & 1) ? 65 : 0] = st.h[m];
  }
}

// Moves a double one lane along the wave (DPP wave shift): SHR gives lane l the
// value of lane l - 1, SHL that of lane l + 1; the lane without a source takes `edge`.
template <bool SHR>
__device__ __forceinline__ double wave_shift(double v, double edge) {
  constexpr int ctrl = SHR ? 0x138 : 0x130;      // wave_shr:1 / wave_shl:1
  const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
  const int lo = __builtin_amdgcn_update_dpp((int)e, (int)b, ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(e >> 32), (int)(b >> 32), ctrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Species wave a adds its reaction populations from the staged records.  For row r
// of directions (c_y, c_z), the lane of node x evaluates at its own record the three
// populations that record sends (to x - 1, x, x + 1 for c_x = -1, 0, +1); the c_x =
// +1 one moves one lane up and the c_x = -1 one one lane down.  Lane 0 takes its
// c_x = +1 population from the record left of the wave and lane 63 its c_x = -1 one
// from the record right of it, evaluated in the same pass (one record per lane).
// A third of the LDS reads of a pull that reads every source record, same products.
template <int D, int M, bool ENERGY>
__device__ __forceinline__ void add_staged_sources(const KParams &p, const SpeciesShared<D, M, ENERGY> &sh, int a,
                                                   int lane, double km, double *f) {
  using SS = SpeciesShared<D, M, ENERGY>;
  constexpr int R = SS::R;
  const int j = lane + 1;
  const bool right = lane == 63;
  const int jh = right ? 65 : 0;                  // the record outside the wave this lane needs
  const double ch = right ? -1.0 : 1.0;           // and the c_x it sends to this lane
#pragma unroll
  for (int r = 0; r < R; ++r) {
    SrcVals<D> v, vh;
    v.sa = sh.u.s.stage[r][a][j];
    v.T = sh.u.s.stage[r][M][j];
    vh.sa = sh.u.s.stage[r][a][jh];
    vh.T = sh.u.s.stage[r][M][jh];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      v.v[d] = sh.u.s.stage[r][M + 1 + d][j];
      vh.v[d] = sh.u.s.stage[r][M + 1 + d][jh];
    }
    const double qm = source_population<D>(v, km, p.inv_T_ref, 3 * r);       // c_x = -1
    const double q0 = source_population<D>(v, km, p.inv_T_ref, 3 * r + 1);   // c_x = 0
    const double qp = source_population<D>(v, km, p.inv_T_ref, 3 * r + 2);   // c_x = +1
    double qh;                                     // source_population with c_x = ch
    {
      const double RaT = km * (vh.T * p.inv_T_ref);
      const double Px = vh.v[0] * vh.v[0] + RaT;
      double psi = vh.sa * (0.5 * (ch * vh.v[0] + Px));
#pragma unroll
      for (int d = 1; d < D; ++d) {
        const double P = vh.v[d] * vh.v[d] + RaT;
        const int c = cdir(3 * r, d);
        psi *= (c == 0) ? 1.0 - P : 0.5 * (c * vh.v[d] + P);
      }
      qh = psi;
    }
    f[3 * r + 1] += q0;
    f[3 * r + 2] += wave_shift<true>(qp, qh);
    f[3 * r] += wave_shift<false>(qm, qh);
  }
}

// Per-node state every wave derives from the lattice moments in LDS.
template <int D, int M>
struct NodeState {
  double rho_a[M], Y[M], RaT[M];
  double rho, u[D], v[D], im, T, RT, Ps;
  double g;                   // 1 / (dfac im): 1/tau_ab = R_a T g / (m_b D_ab^ref)
};

// Reciprocals replace the per-species divisions (fewer dependent chains, fewer
// live registers); the results differ from the divided forms by rounding only.
// jm: first moment of the momentum lattice (phi rho u... = rho u, eq f1momMomentum).
template <int D, int M, bool ENERGY>
__device__ __forceinline__ void node_state(const KParams &p, const SpeciesShared<D, M, ENERGY> &sh, int lane,
                                           const double *jm, double phi, double Tfield, NodeState<D, M> &s) {
  const double iphi = 1.0 / phi;
  s.rho = sh.m0[M][lane] * iphi;
  const double irho = 1.0 / s.rho;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    s.u[d] = jm[d] * irho;
    s.v[d] = s.u[d] * iphi;
  }
  double rs = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    s.rho_a[a] = sh.m0[a][lane] * iphi;
    rs += s.rho_a[a];
  }
  const double irs = 1.0 / rs;
  s.im = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    s.Y[a] = s.rho_a[a] * irs;
    s.im += s.Y[a] * p.inv_m[a];
  }
  if constexpr (ENERGY) {
    const double E = sh.m0[M + 1][lane] * iphi * irho;
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) v2 += s.v[d] * s.v[d];
    double cvm = 0.0, u0m = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      cvm += s.Y[a] * p.cv[a];
      u0m += s.Y[a] * p.uf[a];
    }
    s.T = (E - 0.5 * v2 - u0m) / cvm;                 // eq temperature
  } else {
    s.T = Tfield;
  }
  s.RT = 0.0;
  s.Ps = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    s.RaT[a] = p.theta_ref * p.mmin_over_m[a] * (s.T * p.inv_T_ref);
    s.RT += s.Y[a] * s.RaT[a];
    s.Ps += s.rho_a[a] * s.RaT[a];
  }
  const double Tr = s.T * p.inv_T_ref;
  // D_ab(T, P) = D_ab^ref (T/T_ref)^1.5 / P  ->  1/tau_ab = R_a T P / ((T/T_ref)^1.5 m_b D_ab^ref im)
  s.g = s.Ps / (Tr * sqrt(Tr) * s.im);
}

// Second-order species momenta (eq transform1 with the Knudsen terms): solves
// A x = j from the rows in LDS (Gaussian elimination, M x M) and writes x to LDS.
// The matrix is factored once; the D right-hand sides are then solved one at a
// time in a loop kept rolled, so only one column of momenta is live: this is the
// kernel's register peak, and with it at 156-162 VGPRs three waves fit on a SIMD
// (the two 6-wave tiles of a D3Q27 block).
template <int D, int M, bool ENERGY>
__device__ __forceinline__ void species_momenta(SpeciesShared<D, M, ENERGY> &sh, int lane) {
  double A[M][M];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int c = 0; c < M; ++c) A[a][c] = sh.u.s.A[a][c][lane];
  double inv[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    inv[k] = 1.0 / A[k][k];
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      A[r][k] *= inv[k];                      // multiplier l_rk
#pragma unroll
      for (int c = k + 1; c < M; ++c) A[r][c] -= A[r][k] * A[k][c];
    }
  }
#pragma unroll 1
  for (int d = 0; d < D; ++d) {
    double x[M];
#pragma unroll
    for (int a = 0; a < M; ++a) x[a] = sh.u.s.m1[a][d][lane];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int r = k + 1; r < M; ++r) x[r] -= A[r][k] * x[k];
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
      double sacc = x[k];
#pragma unroll
      for (int c = k + 1; c < M; ++c) sacc -= A[k][c] * x[c];
      x[k] = sacc * inv[k];
    }
#pragma unroll
    for (int a = 0; a < M; ++a) sh.x[a][d][lane] = x[a];
  }
}

// Barrier of the L waves of one tile of a block (the hardware barrier spans the
// whole block): every wave adds one to the tile's LDS counter after its own LDS
// writes and waits until the count reaches `target` (L per barrier so far).  The
// wait is bounded (`polls`, by default 2^18, far beyond any real wait), so every
// wave leaves it; false when it ran out.
__device__ __forceinline__ bool tile_sync(int *cnt, int target, int lane, int polls) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  if (lane == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  bool ok = false;
  for (int spin = 0; spin < polls; ++spin) {
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= target) {
      ok = true;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  return ok;
}

template <int D, int M, bool ENERGY, typename PT, int TB>
__global__ __launch_bounds__(64 * TB * (M + 1 + (ENERGY ? 1 : 0))) void k_species(const KParams p) {
  constexpr int Q = LQ<D>::Q;
  constexpr int L = M + 1 + (ENERGY ? 1 : 0);
  __shared__ SpeciesShared<D, M, ENERGY> shb[TB];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = TB > 1 ? wv / L : 0;                 // tile of the block this wave works on
  const int w = wv - t * L;                          // wave-uniform role (scalar)
  SpeciesShared<D, M, ENERGY> &sh = shb[t];
  const int lane = threadIdx.x & 63;
  // The two tiles of a block synchronise their own waves only, so that one tile's
  // loads overlap the other's serial phases instead of both waiting at every barrier.
  __shared__ int tcnt[TB];
  if constexpr (TB > 1) {
    if (threadIdx.x < TB) tcnt[threadIdx.x] = 0;
    __syncthreads();
  }
  int tphase = 0;
  bool synced = true;
  auto sync = [&]() {
    if constexpr (TB == 1) {
      __syncthreads();
    } else {
      tphase += L;
      synced &= tile_sync(&tcnt[t], tphase, lane, p.tile_polls);
    }
  };
  // Blocks b = 8 k + x run on XCD x (dispatch order).  Each XCD walks its own part
  // of the grid in order, so that a row's staged neighbour records are fetched once
  // into that XCD's L2 and re-read from there: with xcd_slabs, XCD x owns the y slab
  // x of every z plane and walks it z by z (the nine record rows a tile stages lie in
  // three consecutive slab planes); otherwise the x-th eighth of the nodes.
  const unsigned nb = gridDim.x;
  const unsigned b = blockIdx.x;
  unsigned n0;
  if (p.xcd_slabs) {
    const unsigned bpr = (unsigned)p.nx / (64u * TB), rps = (unsigned)p.ny >> 3;
    const unsigned k = b >> 3, r = k / bpr;
    const unsigned y = (b & 7u) * rps + r % rps, z = r / rps;
    n0 = (z * (unsigned)p.ny + y) * (unsigned)p.nx + (k % bpr) * 64u * TB;
  } else {
    n0 = ((b & 7u) * (nb >> 3) + (b >> 3)) * 64u * TB;
  }
  const int n = (int)(n0 + 64u * t) + lane;
  const bool valid = n < p.N;
  const int N = p.N;

  Node nd;
  nd.n = n;
  nd.x = nd.y = nd.z = 0;
  nd.flag = 0;
  double phi = 1.0, Tfield = 0.0;
  double vb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) vb[d] = 0.0;
  bool inlet_node = false;
  PullGeo<D> geo = {};
  if (valid) {
    if (p.colflag) {
      nd.flag = p.colflag[n];
    } else {
      nd.x = n % p.nx;
      const int r = n / p.nx;
      nd.y = r % p.ny;
      nd.z = r / p.ny;
      nd.flag = (nd.x == 0 ? 1 : 0) | (nd.x == p.nx - 1 ? 2 : 0);
    }
    phi = p.phi[n];
    if (!ENERGY) Tfield = p.Tfield[n];
    inlet_node = is_inlet_node(p, nd);
    geo = pull_geo<D>(p, nd);
    if (inlet_node) {
#pragma unroll
      for (int d = 0; d < D; ++d) vb[d] = p.rec_prev[(size_t)d * N + n];
    }
  }

  // ---- phase 1: pull this wave's lattice (species a, momentum M, energy M + 1)
  //      with the previous step's reaction populations, moments to LDS
  const int lat = w;
  const bool rows = p.src_prev && row_block<D>(p, nd, geo, valid);   // the same in every wave of the tile
  Stage<D, M, ENERGY> st;
  if (rows) load_stage<D, M, ENERGY>(p, nd, w, lane, st);
  double f[Q];
  if (valid) pull_populations<D, PT>(p, nd, geo, lat, f);
  if (p.src_prev) {
    if (rows) store_stage<D, M, ENERGY>(w, lane, st, sh);
    sync();
    if (valid && lat < M) {
      const double km = species_km<M>(p, lat);
      if (rows)
        add_staged_sources<D, M, ENERGY>(p, sh, lat, lane, km, f);
      else
        add_source_populations<D>(p, nd, geo, p.rec_prev + (size_t)(kRecSrc + lat) * N, km, f);
    }
  }
  if (valid) {
    if (inlet_node) inlet_replace<D, M>(p, nd, lat, phi, vb, f);
    double s0 = 0.0, s1[D];
#pragma unroll
    for (int d = 0; d < D; ++d) s1[d] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s0 += f[i];
#pragma unroll
      for (int d = 0; d < D; ++d) s1[d] += cdir(i, d) * f[i];
    }
    sh.m0[lat][lane] = s0;
    if (lat <= M) {
#pragma unroll
      for (int d = 0; d < D; ++d) sh.u.s.m1[lat][d][lane] = s1[d];
    }
  }
  sync();

  // ---- phase 2: node state; species wave a publishes its rates and its row
  NodeState<D, M> s;
  double iab[M], beta = 0.0, itk_a = 0.0, RaTa = 0.0, Ya = 0.0;
  if (valid && w < M) {
    {
      double jm[D];
#pragma unroll
      for (int d = 0; d < D; ++d) jm[d] = sh.u.s.m1[M][d][lane];
      node_state<D, M, ENERGY>(p, sh, lane, jm, phi, Tfield, s);
    }
    {
      const int a = w;
#pragma unroll
      for (int c = 0; c < M; ++c) {              // select without indexing by the run-time a
        if (c == a) { RaTa = s.RaT[c]; Ya = s.Y[c]; }
      }
      const double rg = RaTa * s.g;
      double it = 0.0;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        iab[c] = (c != a) ? rg * p.imD[a * LBM_MMAX + c] : 0.0;   // 1/tau_ab (eq tauab)
        it += s.Y[c] * iab[c];
      }
      beta = it / (2.0 + it);                   // eq betaa
      itk_a = p.knudsen ? sqrt(RaTa) / p.kfac[n] : 0.0;   // eq tauak: R_a T / (kfac sqrt(R_a T))
#pragma unroll
      for (int c = 0; c < M; ++c)
        sh.u.s.A[a][c][lane] = (c == a) ? 1.0 + 0.5 * it + 0.5 * itk_a : -0.5 * Ya * iab[c];
      sh.u.s.itk[a][lane] = itk_a;
    }
  }
  sync();

  if (w < M) {
    // ---- species wave a: waits for the second-order momenta of the momentum
    //      wave, publishes Delta_a,i = phi rho_a (Psi_i(v, R_a T) - Psi_i(xi_a, R_a T)),
    //      then collides (eqs 27eq, 27qeq, fKnudsen, fStar,
    //      finalNumericalEquationsReactive) with the cross term
    //      sum_{c != a} (1/tau_ac) Delta_c,i read back from LDS.
    const int a = w;
    sync();                              // x is in LDS; m1, A, itk are free
    double te[D][3], ts[D][3], tk[D][3];
    const double pra = sh.m0[a][lane];            // phi rho_a
    const bool pos = pra > 0.0;
    const double ipra = pos ? 1.0 / pra : 0.0;
    if (valid) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double xs = sh.x[a][d][lane] * ipra;   // j_a / (phi rho_a), 0 when rho_a = 0
        const double Pe = s.v[d] * s.v[d] + RaTa, Ps = xs * xs + RaTa;
        te[d][0] = 0.5 * (-s.v[d] + Pe); te[d][1] = 1.0 - Pe; te[d][2] = 0.5 * (s.v[d] + Pe);
        ts[d][0] = 0.5 * (-xs + Ps);     ts[d][1] = 1.0 - Ps; ts[d][2] = 0.5 * (xs + Ps);
        tk[d][0] = 0.5 * RaTa;           tk[d][1] = 1.0 - RaTa; tk[d][2] = 0.5 * RaTa;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        double pe = te[0][i % 3], ps = ts[0][i % 3];
        if (D > 1) { pe *= te[1][(i / 3) % 3]; ps *= ts[1][(i / 3) % 3]; }
        if (D > 2) { pe *= te[2][i / 9]; ps *= ts[2][i / 9]; }
        sh.u.dlt[a][i][lane] = pra * (pe - ps);
      }
    }
    sync();
    if (valid) {
      const size_t o = (size_t)(a * Q) * N + n;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        double F = 0.0;                            // iab[a] == 0: the own term drops out
#pragma unroll
        for (int c = 0; c < M; ++c) F += iab[c] * sh.u.dlt[c][i][lane];
        double pe = te[0][i % 3], ps = ts[0][i % 3], pk = tk[0][i % 3];
        if (D > 1) { pe *= te[1][(i / 3) % 3]; ps *= ts[1][(i / 3) % 3]; pk *= tk[1][(i / 3) % 3]; }
        if (D > 2) { pe *= te[2][i / 9]; ps *= ts[2][i / 9]; pk *= tk[2][i / 9]; }
        const double feq = pra * pe;
        const double fst = pos ? pra * ps : 0.0;
        const double fk = pra * pk;
        const double Fi = Ya * F + itk_a * (fst - fk);
        const double f0 = f[i];
        double fo = f0 + 2.0 * beta * (feq - f0) + (beta - 1.0) * Fi;
        if (i == 0 && !synced) fo = __builtin_nan("");   // a tile wait ran out: fail the health check
        store_pop<PT>(p.pout, o + (size_t)i * N, fo);
      }
    }
  } else if (w == M) {
    // ---- momentum wave: solves the species-momentum system and publishes the
    //      second-order momenta; after the barrier that releases the species
    //      waves it rebuilds the node state and writes the node records for the
    //      chemistry and mixture kernels and for the next step.
    double jm[D], itk[M];
    if (valid) {
      species_momenta<D, M, ENERGY>(sh, lane);
#pragma unroll
      for (int c = 0; c < M; ++c) itk[c] = sh.u.s.itk[c][lane];
#pragma unroll
      for (int d = 0; d < D; ++d) jm[d] = sh.u.s.m1[M][d][lane];
    }
    sync();                              // x in LDS; the union now belongs to the species waves
    if (valid) {
      node_state<D, M, ENERGY>(p, sh, lane, jm, phi, Tfield, s);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        double fk = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) fk -= sh.x[c][d][lane] * itk[c];   // eq netKnudsenForce
        __builtin_nontemporal_store(                 // rho u (1 - 3RT) - rho u^3 / phi^2, with v = u / phi
            s.rho * s.u[d] * (1.0 - 3.0 * s.RT) - s.rho * s.u[d] * s.v[d] * s.v[d], p.rA + (size_t)d * N + n);
        if (p.knudsen) __builtin_nontemporal_store(fk, p.rFk + (size_t)d * N + n);
        if (p.need_v) __builtin_nontemporal_store(s.v[d], p.rec_cur + (size_t)d * N + n);
      }
      __builtin_nontemporal_store(s.RT, p.rRT + n);
      if (p.chem) {
#pragma unroll
        for (int a = 0; a < M; ++a) __builtin_nontemporal_store(s.rho_a[a], p.rrho + (size_t)a * N + n);
      }
      if constexpr (ENERGY) {
        p.T_cur[n] = s.T;
        // inlet node: the state the next step's entering energy populations take
        // (the node's mixture at the inlet temperature)
        const int side = ((nd.flag & 1) && p.bc_lo == BC_INLET) ? 0 : (((nd.flag & 2) && p.bc_hi == BC_INLET) ? 1 : -1);
        if (side >= 0) {
          const double Tin = side == 0 ? p.inlet[0].T_K : p.inlet[1].T_K;
          double Ui = 0.0, RTi = 0.0;
#pragma unroll
          for (int a = 0; a < M; ++a) {
            Ui += s.Y[a] * (p.uf[a] + p.cv[a] * Tin);
            RTi += s.Y[a] * (p.theta_ref * p.mmin_over_m[a] * (Tin * p.inv_T_ref));
          }
          double *e = p.rec_cur + (size_t)kRecEin * N + n;
          e[0] = s.rho;
          e[N] = Ui;
          e[2 * (size_t)N] = RTi;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
          double ub = 0.0;
#pragma unroll
          for (int c = 0; c < M; ++c)
            ub += s.Y[c] * ((s.rho_a[c] > 0.0) ? sh.x[c][d][lane] / s.rho_a[c] : s.u[d]);
          double sacc = 0.0;
#pragma unroll
          for (int a = 0; a < M; ++a) {
            const double ua = (s.rho_a[a] > 0.0) ? sh.x[a][d][lane] / s.rho_a[a] : s.u[d];
            const double Ha = p.uf[a] + p.cv[a] * s.T + s.RaT[a];
            sacc += Ha * s.Y[a] * (ua - ub);
          }
          p.rqd[(size_t)d * N + n] = sacc;
        }
        double yu = 0.0, yc = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
          p.rY[(size_t)a * N + n] = s.Y[a];
          yu += p.uf[a] * s.Y[a];
          yc += (p.cv[a] + p.theta_ref * p.mmin_over_m[a] * p.inv_T_ref) * s.Y[a];
        }
        p.rY[(size_t)M * N + n] = yu;           // H_a(T) = uf_a + (cv_a + R_a/T) T: the stencil of
        p.rY[(size_t)(M + 1) * N + n] = yc;     // sum_a H_a(T_x) Y_a needs two fields, not M
      }
    }
    sync();
  } else {
    sync();                              // energy wave: nothing after its pull
    sync();
  }
}

// ---------------------------------------------------------------------------
// k_species_lane: k_species for one-dimensional lattices without the energy
// lattice, one node per lane.  With three directions per lattice a node's whole
// species step (its six pulls, moments, rates, the M x M solve and the M
// collisions) fits one lane, so the 64 nodes of a tile need one wave instead of
// M + 1, no barrier and no LDS; on the batched 1-D columns the tile kernel's
// waves take several rounds of the chip, this one a single round.  The
// arithmetic is k_species' in the same order; the values that kernel hands
// between waves through LDS pass through an empty asm here, so the compiler
// forms the same fused multiply-adds and the results are the same bitwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int M, typename PT>
__global__ __launch_bounds__(256) void k_species_lane(const KParams p) {
  constexpr int D = 1, Q = 3;
  Node nd;
  if (!get_node(p, nd)) return;
  const int N = p.N;
  const int n = nd.n;
  const double phi = p.phi[n];
  const double Tfield = p.Tfield[n];
  const bool inlet_node = is_inlet_node(p, nd);
  double vb[D];
  vb[0] = inlet_node ? p.rec_prev[n] : 0.0;
  const PullGeo<D> geo = pull_geo<D>(p, nd);

  // ---- pull every lattice with the previous step's reaction populations; moments
  double f[M + 1][Q], m0[M + 1], m1[M + 1];
#pragma unroll
  for (int l = 0; l <= M; ++l) pull_populations<D, PT>(p, nd, geo, l, f[l]);
#pragma unroll
  for (int l = 0; l <= M; ++l) {
    if (l < M && p.src_prev)
      add_source_populations<D>(p, nd, geo, p.rec_prev + (size_t)(kRecSrc + l) * N, species_km<M>(p, l), f[l]);
    if (inlet_node) inlet_replace<D, M>(p, nd, l, phi, vb, f[l]);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s0 += f[l][i];
      s1 += cdir(i, 0) * f[l][i];
    }
    m0[l] = lane_opaque(s0);
    m1[l] = lane_opaque(s1);
  }

  // ---- node state (as node_state)
  const double iphi = 1.0 / phi;
  const double rho = m0[M] * iphi;
  const double irho = 1.0 / rho;
  const double u = m1[M] * irho;
  const double v = u * iphi;
  double rho_a[M], rs = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    rho_a[a] = m0[a] * iphi;
    rs += rho_a[a];
  }
  const double irs = 1.0 / rs;
  double Y[M], RaT[M], im = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Y[a] = rho_a[a] * irs;
    im += Y[a] * p.inv_m[a];
  }
  double RT = 0.0, Ps = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    RaT[a] = p.theta_ref * p.mmin_over_m[a] * (Tfield * p.inv_T_ref);
    RT += Y[a] * RaT[a];
    Ps += rho_a[a] * RaT[a];
  }
  const double Tr = Tfield * p.inv_T_ref;
  const double g = Ps / (Tr * sqrt(Tr) * im);

  // ---- rates and rows of the species-momentum system (eqs tauab, betaa, tauak, transform1)
  double iab[M][M], beta[M], itk[M], A[M][M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double RaTa = lane_opaque(RaT[a]), Ya = lane_opaque(Y[a]);   // selected per wave in k_species
    const double rg = RaTa * g;
    double it = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      iab[a][c] = lane_opaque((c != a) ? rg * p.imD[a * LBM_MMAX + c] : 0.0);
      it += Y[c] * iab[a][c];
    }
    beta[a] = it / (2.0 + it);
    itk[a] = p.knudsen ? sqrt(RaTa) / p.kfac[n] : 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c)
      A[a][c] = lane_opaque((c == a) ? 1.0 + 0.5 * it + 0.5 * itk[a] : -0.5 * Ya * iab[a][c]);
  }
  // ---- second-order species momenta (as species_momenta)
  double inv[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    inv[k] = 1.0 / A[k][k];
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      A[r][k] *= inv[k];
#pragma unroll
      for (int c = k + 1; c < M; ++c) A[r][c] -= A[r][k] * A[k][c];
    }
  }
  double x[M];
#pragma unroll
  for (int a = 0; a < M; ++a) x[a] = m1[a];
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int r = k + 1; r < M; ++r) x[r] -= A[r][k] * x[k];
#pragma unroll
  for (int k = M - 1; k >= 0; --k) {
    double sacc = x[k];
#pragma unroll
    for (int c = k + 1; c < M; ++c) sacc -= A[k][c] * x[c];
    x[k] = lane_opaque(sacc * inv[k]);
  }

  // ---- node records (as the momentum wave of k_species)
  {
    double fk = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) fk -= x[c] * lane_opaque(itk[c]);   // eq netKnudsenForce
    __builtin_nontemporal_store(rho * u * (1.0 - 3.0 * RT) - rho * u * v * v, p.rA + n);
    if (p.knudsen) __builtin_nontemporal_store(fk, p.rFk + n);
    if (p.need_v) __builtin_nontemporal_store(v, p.rec_cur + n);
    __builtin_nontemporal_store(RT, p.rRT + n);
    if (p.chem) {
#pragma unroll
      for (int a = 0; a < M; ++a) __builtin_nontemporal_store(rho_a[a], p.rrho + (size_t)a * N + n);
    }
  }

  // ---- species collision (eqs 27eq, 27qeq, fKnudsen, fStar, finalNumericalEquationsReactive)
  double te[M][Q], ts[M][Q], dlt[M][Q];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double RaTa = lane_opaque(RaT[a]);
    const double pra = m0[a];
    const bool pos = pra > 0.0;
    const double ipra = pos ? 1.0 / pra : 0.0;
    const double xs = x[a] * ipra;
    const double Pe = v * v + RaTa, Pst = xs * xs + RaTa;
    te[a][0] = 0.5 * (-v + Pe); te[a][1] = 1.0 - Pe; te[a][2] = 0.5 * (v + Pe);
    ts[a][0] = 0.5 * (-xs + Pst); ts[a][1] = 1.0 - Pst; ts[a][2] = 0.5 * (xs + Pst);
#pragma unroll
    for (int i = 0; i < Q; ++i) dlt[a][i] = lane_opaque(pra * (te[a][i] - ts[a][i]));
  }
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double RaTa = lane_opaque(RaT[a]), Ya = lane_opaque(Y[a]);
    const double pra = m0[a];
    const bool pos = pra > 0.0;
    const double tk[Q] = {0.5 * RaTa, 1.0 - RaTa, 0.5 * RaTa};
    const size_t o = (size_t)(a * Q) * N + n;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double F = 0.0;
#pragma unroll
      for (int c = 0; c < M; ++c) F += iab[a][c] * dlt[c][i];
      const double feq = pra * te[a][i];
      const double fst = pos ? pra * ts[a][i] : 0.0;
      const double fkn = pra * tk[i];
      const double Fi = Ya * F + itk[a] * (fst - fkn);
      const double f0 = f[a][i];
      store_pop<PT>(p.pout, o + (size_t)i * N, f0 + 2.0 * beta[a] * (feq - f0) + (beta[a] - 1.0) * Fi);
    }
  }
}

// ---------------------------------------------------------------------------
// k_mixture: momentum lattice with the extended equilibrium, energy lattice
// ---------------------------------------------------------------------------
template <int D, int M, bool ENERGY, typename PT>
__global__ __launch_bounds__(256) void k_mixture(const KParams p) {
  constexpr int Q = LQ<D>::Q;
  Node nd;
  if (!get_node(p, nd)) return;
  const int N = p.N;
  const int n = nd.n;
  const double phi = p.phi[n];
  double vb[D];
  const bool inlet_node = is_inlet_node(p, nd);
#pragma unroll
  for (int d = 0; d < D; ++d) vb[d] = inlet_node ? p.rec_prev[(size_t)d * N + n] : 0.0;
  const PullGeo<D> geo = pull_geo<D>(p, nd);

  double f[Q];
  pull_lattice<D, M, true, PT>(p, nd, geo, M, phi, vb, inlet_node, f);
  double sf = 0.0, jf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) jf[d] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    sf += f[i];
#pragma unroll
    for (int d = 0; d < D; ++d) jf[d] += cdir(i, d) * f[i];
  }
  const double rho = sf / phi;
  double u[D], v[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[d] = jf[d] / rho;
    v[d] = u[d] / phi;
  }
  const double RT = p.rRT[n];
  const double omega = 1.0 / (p.nu / RT + 0.5);

  // Galilean correction: G_a = d_a (rho u_a (1 - 3RT) - rho u_a^3 / phi^2), isotropic stencil
  double G[D];
#pragma unroll
  for (int d = 0; d < D; ++d) G[d] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (cnorm2<D>(i) == 0) continue;
    const int m = nb_node<D>(p, nd, i);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int c = cdir(i, d);
      if (c != 0) G[d] += wdir<D>(i) * c * p.rA[(size_t)d * N + m];
    }
  }
  double Pex[D], xi[D];
  const double gfac = (2.0 - omega) / (2.0 * phi * rho * omega);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    G[d] *= 3.0;
    Pex[d] = RT + v[d] * v[d] + gfac * G[d];
    const double Fk = p.knudsen ? p.rFk[(size_t)d * N + n] : 0.0;
    xi[d] = (u[d] + Fk / (omega * rho)) / phi;          // u^ex / phi
  }
  const double ratio = p.chem ? p.srcsum_cur[n] / (phi * rho) : 0.0;   // rho_pc / rho - 1
  const double phirho = phi * rho;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double fex = phirho * psi_dir<D>(i, xi, Pex);
    store_pop<PT>(p.pout, (size_t)(M * Q + i) * N + n, f[i] + omega * (fex - f[i]) + ratio * fex);
  }

  if (ENERGY) {
    // second moment of the pre-collision momentum populations
    double Pab[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) Pab[a][b] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) Pab[a][b] += (cdir(i, a) * cdir(i, b)) * f[i];
    const double T = p.T_cur[n];
    double Y[M], Ha[M];
    double U = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      Y[a] = p.rY[(size_t)a * N + n];
      const double Ua = p.uf[a] + p.cv[a] * T;
      U += Y[a] * Ua;
      Ha[a] = Ua + p.theta_ref * p.mmin_over_m[a] * (T * p.inv_T_ref);
    }
    const double Hmix = U + RT;
    const double P = rho * RT;
    const double omega1 = 1.0 / (p.nu / (p.prandtl * RT) + 0.5);
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) v2 += v[d] * v[d];
    // sum_a H_a d_a Y_a (isotropic stencil on the mass fractions)
    double four[D];
#pragma unroll
    for (int d = 0; d < D; ++d) four[d] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cnorm2<D>(i) == 0) continue;
      const int m = nb_node<D>(p, nd, i);
      const double hy = p.rY[(size_t)M * N + m] + T * p.rY[(size_t)(M + 1) * N + m];   // sum_a H_a(T) Y_a(m)
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int c = cdir(i, d);
        if (c != 0) four[d] += wdir<D>(i) * c * hy;
      }
    }
    double g[Q], q[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q[d] = 0.0;
    pull_lattice<D, M, true, PT>(p, nd, geo, M + 1, phi, vb, inlet_node, g);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
#pragma unroll
      for (int d = 0; d < D; ++d) q[d] += cdir(i, d) * g[i];
    }
    // Q_a = (omega - omega1) (q* - q^eq), expanded (eqs gstareq1mom, interdiffusion,
    //       corrFourier, qex; natural bulk viscosity)
    double Qv[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double qeq = rho * u[a] * (Hmix + 0.5 * v2);
      double corr = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const double Peq = phirho * v[a] * v[b] + (a == b ? phi * P : 0.0);
        corr += v[b] * (Pab[a][b] - Peq);
      }
      const double qd = p.rqd[(size_t)a * N + n];
      Qv[a] = (omega - omega1) * (q[a] - qeq - corr) + omega1 * rho * qd +
              0.5 * (2.0 - omega1) * P * phi * (3.0 * four[a]) - 0.5 * (omega - omega1) * v[a] * G[a];
    }
    // chemistry (eqs temperatureCell, InternalEnergyCell_PC, g0mom_source,
    // g_source): the unified internal energy of fluid and adsorbed phase at
    // this T is kept, phi rho^pc U^pc = phi rho U + E_s(before) - E_s(after);
    // g^eq,source is g^eq with (rho^pc, U^pc) at the pre-collision v and RT
    double phirho_pc = phirho, U_pc = U;
    if (p.chem) {
      phirho_pc = phirho + p.srcsum_cur[n];
      double dEs = 0.0;
      if (p.esrc) {
        double es = 0.0;
        for (int k = 0; k < p.K; ++k) es += p.theta[(size_t)k * N + n] * (p.es_u[k] + p.es_c[k] * T);
        dEs = p.rEs[n] - es;
      }
      if (p.uel) dEs += p.uel[n];               // the electrical source joins the unified energy
      U_pc = (phirho * U + dEs) / phirho_pc;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double ge = geq_dir<D>(i, phirho, U, RT, v);
      double out = g[i] + omega * (ge - g[i]);
      if (p.chem) out += geq_dir<D>(i, phirho_pc, U_pc, RT, v) - ge;   // eq g_source
      if (cnorm2<D>(i) == 1) {
        double cq = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) cq += cdir(i, d) * Qv[d];
        out += 0.5 * cq;
      }
      store_pop<PT>(p.pout, (size_t)((M + 1) * Q + i) * N + n, out);
    }
  }
}

// ---------------------------------------------------------------------------
// moments kernel: macroscopic fields at the current time level
// ---------------------------------------------------------------------------
template <int D, int M, bool ENERGY, typename PT>
__global__ __launch_bounds__(256) void k_moments(const KParams p, double *out) {
  Node nd;
  if (!get_node(p, nd)) return;
  const int N = p.N;
  const int n = nd.n;
  const double phi = p.phi[n];
  SpeciesState<D, M> S;
  species_front<D, M, ENERGY, PT>(p, nd, phi, S);
  size_t r = 0;
  double rs = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) out[(r++) * N + n] = S.rho_a[a];
#pragma unroll
  for (int d = 0; d < D; ++d) out[(r++) * N + n] = S.u[d];
  out[(r++) * N + n] = S.T;
  out[(r++) * N + n] = S.rho * S.RT;
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) out[(r++) * N + n] = S.ja[a][d];
  out[(r++) * N + n] = S.rho;
#pragma unroll
  for (int a = 0; a < M; ++a) rs += S.Y[a] * p.inv_m[a];
#pragma unroll
  for (int a = 0; a < M; ++a) out[(r++) * N + n] = (S.Y[a] * p.inv_m[a]) / rs;
}

// ---------------------------------------------------------------------------
// initial equilibria at zero velocity (stored post-stream)
// ---------------------------------------------------------------------------
template <int D, int M, typename PT>
__global__ __launch_bounds__(256) void k_init(const InitParams ip) {
  constexpr int Q = LQ<D>::Q;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ip.N) return;
  const int N = ip.N;
  const double phi = ip.phi[n];
  const double T = ip.T0[n];
  const double Pl = ip.Plat[n];
  double rho_a[M], RaT[M];
  double rho = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    RaT[a] = ip.theta_ref * ip.mmin_over_m[a] * (T * ip.inv_T_ref);
    rho_a[a] = ip.X0[(size_t)a * N + n] * Pl / RaT[a];     // P_a = X_a P = rho_a R_a T
    rho += rho_a[a];
  }
  double RT = 0.0, U = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double Y = rho_a[a] / rho;
    RT += Y * RaT[a];
    U += Y * (ip.uf[a] + ip.cv[a] * T);
  }
  const double zero[3] = {0.0, 0.0, 0.0};
  PT *pop = static_cast<PT *>(ip.pop);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const double Pa[3] = {RaT[a], RaT[a], RaT[a]};
      pop[(size_t)(a * Q + i) * N + n] = (PT)(phi * rho_a[a] * psi_dir<D>(i, zero, Pa));
    }
    const double Pm[3] = {RT, RT, RT};
    pop[(size_t)(M * Q + i) * N + n] = (PT)(phi * rho * psi_dir<D>(i, zero, Pm));
    if (ip.energy) pop[(size_t)((M + 1) * Q + i) * N + n] = (PT)geq_dir<D>(i, phi * rho, U, RT, zero);
  }
}

// ---------------------------------------------------------------------------
// Surface chemistry (Section 4): backward Euler on gas concentrations and
// coverages, Newton with dense LU (partial pivoting), extent-based update.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ipow(double x, int e) {
  return e == 0 ? 1.0 : (e == 1 ? x : (e == 2 ? x * x : x * x * x));
}

// Newton unknowns: the M gas concentrations and the K-1 non-vacancy coverages.
// The vacancy follows from site conservation, theta_V = 1 - sum_s theta_s, which
// every site-balanced reaction preserves; Newton on this reduced system gives
// the same iterates as Newton on all M+K unknowns started on the balanced set.
// One node per lane: the U x U FP64 Jacobian lives in registers (occupancy 1);
// each reaction's stoichiometric row is read once as 16 packed coefficients.

// Stoichiometric row of one reaction, 16 coefficients packed in 4 words.
struct NuRow {
  uint32_t w[4];
};
__device__ __forceinline__ NuRow load_nu(const int8_t *row) {
  const uint4 v = *reinterpret_cast<const uint4 *>(row);
  NuRow r;
  r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
  return r;
}
// coefficient of species s (compile-time s after unrolling)
__device__ __forceinline__ int nu_of(const NuRow &r, int s) {
  return (int)((r.w[s >> 2] >> (8 * (s & 3))) & 0xffu);
}

// Rate q = kf prod C^nu_f - kb prod C^nu_b and, when dq != nullptr, dq/dC_t for
// every species (branches are on the reaction's coefficients, uniform per wave).
template <int S>
__device__ __forceinline__ double mass_action(const NuRow &NF, const NuRow &NB, double kf, double kb,
                                              const double *C, double *dq) {
  double pf = kf, pb = kb;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int ef = nu_of(NF, s), eb = nu_of(NB, s);
    if (ef) pf *= ipow(C[s], ef);
    if (eb) pb *= ipow(C[s], eb);
  }
  if (dq) {
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int ft = nu_of(NF, t), bt = nu_of(NB, t);
      double d = 0.0;
      if (ft) {
        double df = kf * ft * ipow(C[t], ft - 1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int e = nu_of(NF, s);
          if (s != t && e) df *= ipow(C[s], e);
        }
        d += df;
      }
      if (bt) {
        double db = kb * bt * ipow(C[t], bt - 1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int e = nu_of(NB, s);
          if (s != t && e) db *= ipow(C[s], e);
        }
        d -= db;
      }
      dq[t] = d;
    }
  }
  return pf - pb;
}

template <int M, int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_chem(const ChemParams cp) {
  constexpr int S = M + K;      // unknowns: gas concentrations and every coverage (vacancies too)
  __shared__ double s_k[2 * LBM_RMAX][64];    // kf, kb of every reaction at this lane's node
  const int lane = threadIdx.x;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cp.N) return;        // no block barrier below: early exit is safe
  const int N = cp.N;
  const double T = cp.T[n];
  const double phi = cp.phi[n];
  const double h = cp.dt / cp.n_sub;
  const double inv_RT = 1.0 / (cp.R_U * T);
  const ChemTables *__restrict__ tb = cp.tab;
  // charge transfer: z F dPhi / (R_U T) with dPhi = Phi_electrode - Phi_electrolyte
  const double fpot = cp.pel ? cp.F_C * (cp.ped[n] - cp.pel[n]) * inv_RT : 0.0;
  for (int r = 0; r < cp.R; ++r) {
    double kf = tb->A_f[r] * exp(-tb->Ea_f[r] * inv_RT);
    double kb = tb->A_b[r] * exp(-tb->Ea_b[r] * inv_RT);
    const int z = tb->charge_z[r];
    if (z) {                    // Butler-Volmer factors of the mass-action constants
      kf *= exp(tb->beta_ct[r] * z * fpot);
      kb *= exp(-(1.0 - tb->beta_ct[r]) * z * fpot);
    }
    s_k[2 * r][lane] = kf;
    s_k[2 * r + 1][lane] = kb;
  }
  double iv = 0.0;              // charge released per unit volume over the step / dt
  double gk[K];                 // site density of each coverage's surface phase
#pragma unroll
  for (int k = 0; k < K; ++k) gk[k] = tb->gam_k[k];
  double y0[S];
#pragma unroll
  for (int a = 0; a < M; ++a) y0[a] = cp.rrho[(size_t)a * N + n] * cp.rho_unit / cp.m[a];
#pragma unroll
  for (int k = 0; k < K; ++k) y0[M + k] = cp.theta[(size_t)k * N + n];
  double src[M];
#pragma unroll
  for (int a = 0; a < M; ++a) src[a] = 0.0;

  for (int sub = 0; sub < cp.n_sub; ++sub) {
    double y[S];
#pragma unroll
    for (int u = 0; u < S; ++u) y[u] = y0[u];
    for (int it = 0; it < cp.n_newton; ++it) {
      double C[S];
#pragma unroll
      for (int a = 0; a < M; ++a) C[a] = y[a];
#pragma unroll
      for (int k = 0; k < K; ++k) C[M + k] = gk[k] * y[M + k];
      // Newton system divided row-wise by the phase weight (phi, Gamma_k):
      //   J = I - (h / W) sum_r wt_rs st_rs dq_r/dy,  b = -(y - y0) + (h / W) sum_r wt_rs st_rs q_r
      double J[S][S], b[S];
#pragma unroll
      for (int u = 0; u < S; ++u) {
        b[u] = -(y[u] - y0[u]);
#pragma unroll
        for (int v = 0; v < S; ++v) J[u][v] = (u == v) ? 1.0 : 0.0;
      }
      for (int r = 0; r < cp.R; ++r) {
        const NuRow NF = load_nu(tb->nu_f[r]), NB = load_nu(tb->nu_b[r]);
        const int kind = tb->kind[r];
        // gas rows: a^(s) of the reaction's surface, phi for a homogeneous reaction;
        // coverage rows: 1, l_TPB / a^(s)_k for a TPB edge reaction
        const double wg = (kind == 1 ? phi : tb->w_r[r]) * h / phi;
        double dq[S];
        const double q = mass_action<S>(NF, NB, s_k[2 * r][lane], s_k[2 * r + 1][lane], C, dq);
#pragma unroll
        for (int k = 0; k < K; ++k) dq[M + k] *= gk[k];   // dC_k / dtheta_k = Gamma_k
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const int st = nu_of(NB, u) - nu_of(NF, u);
          if (st) {
            const double coef = st * ((u < M) ? wg
                                              : h / gk[u - M] * (kind == 2 ? tb->l_tpb / tb->a_k[u - M] : 1.0));
            b[u] += coef * q;
#pragma unroll
            for (int v = 0; v < S; ++v) J[u][v] -= coef * dq[v];
          }
        }
      }
      // LU with partial pivoting on the equilibrated rows (first maximum on ties)
#pragma unroll
      for (int k = 0; k < S; ++k) {
        int piv = k;
        double amax = fabs(J[k][k]);
#pragma unroll
        for (int r = k + 1; r < S; ++r) {
          const double av = fabs(J[r][k]);
          if (av > amax) { amax = av; piv = r; }
        }
#pragma unroll
        for (int r = k + 1; r < S; ++r) {
          const bool sw = (piv == r);
#pragma unroll
          for (int c = k; c < S; ++c) {
            const double tk = J[k][c];
            J[k][c] = sw ? J[r][c] : tk;
            J[r][c] = sw ? tk : J[r][c];
          }
          const double tbb = b[k];
          b[k] = sw ? b[r] : tbb;
          b[r] = sw ? tbb : b[r];
        }
        const double inv = 1.0 / J[k][k];
#pragma unroll
        for (int r = k + 1; r < S; ++r) {
          const double l = J[r][k] * inv;
#pragma unroll
          for (int c = k + 1; c < S; ++c) J[r][c] -= l * J[k][c];
          b[r] -= l * b[k];
        }
      }
#pragma unroll
      for (int k = S - 1; k >= 0; --k) {
        double sacc = b[k];
#pragma unroll
        for (int c = k + 1; c < S; ++c) sacc -= J[k][c] * b[c];
        b[k] = sacc / J[k][k];
      }
#pragma unroll
      for (int u = 0; u < S; ++u) y[u] += b[u];
    }
    // extents at the implicit state, conservative update of every phase
    double C[S];
#pragma unroll
    for (int a = 0; a < M; ++a) C[a] = y[a];
#pragma unroll
    for (int k = 0; k < K; ++k) C[M + k] = gk[k] * y[M + k];
    double dn[S];                 // gas: mol per m^3 of REV; coverages: mol per m^2 of their surface
#pragma unroll
    for (int u = 0; u < S; ++u) dn[u] = 0.0;
    double ze = 0.0;              // sum_r z_r xi_r: electrons per unit TPB length
    for (int r = 0; r < cp.R; ++r) {
      const NuRow NF = load_nu(tb->nu_f[r]), NB = load_nu(tb->nu_b[r]);
      const int kind = tb->kind[r];
      const double dxi = h * mass_action<S>(NF, NB, s_k[2 * r][lane], s_k[2 * r + 1][lane], C, nullptr);
      ze += tb->charge_z[r] * dxi;
      const double wgas = kind == 1 ? phi : tb->w_r[r];
#pragma unroll
      for (int u = 0; u < S; ++u) {
        const int st = nu_of(NB, u) - nu_of(NF, u);
        if (st)
          dn[u] += st * dxi * ((u < M) ? wgas : (kind == 2 ? tb->l_tpb / tb->a_k[u - M] : 1.0));
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) y0[M + k] += dn[M + k] / gk[k];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      y0[a] += dn[a] / phi;
      src[a] += dn[a] * cp.m[a] / cp.rho_unit;
    }
    iv += cp.F_C * tb->l_tpb * ze / cp.dt;   // eq volumetricCurrent
  }
  if (cp.iv) cp.iv[n] = iv;
  if (cp.dry) return;           // a trial of the current control: only the current is wanted
  if (cp.uel) {                 // electrical work out, ohmic heat in (eqs for P_elec, P_Omega, U_source)
    const double p_elec = fabs(cp.ped[n] - cp.pel[n]) * iv;
    const double p_om = (cp.a_el / tb->l_tpb) * iv * iv * cp.omega[n] * cp.dx;
    cp.uel[n] = (p_om - p_elec) * cp.dt * cp.inv_e_unit;
  }
  if (cp.faradaic) {
    const double r = cp.faradaic[n] * cp.dt;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      if (a == cp.fuel) src[a] -= r * cp.m[a] / cp.rho_unit;
      if (a == cp.product) src[a] += r * cp.m[a] / cp.rho_unit;
    }
  }
  double ssum = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    cp.rec[(size_t)(kRecSrc + a) * cp.N + n] = src[a];
    ssum += src[a];
  }
  cp.srcsum[n] = ssum;
#pragma unroll
  for (int k = 0; k < K; ++k) cp.theta[(size_t)k * N + n] = y0[M + k];
}

// Faradaic source only (no mechanism installed).
template <int M>
__global__ __launch_bounds__(256) void k_faradaic(const ChemParams cp) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cp.N) return;
  const double r = cp.faradaic[n] * cp.dt;
  double ssum = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double s = 0.0;
    if (a == cp.fuel) s -= r * cp.m[a] / cp.rho_unit;
    if (a == cp.product) s += r * cp.m[a] / cp.rho_unit;
    cp.rec[(size_t)(kRecSrc + a) * cp.N + n] = s;
    ssum += s;
  }
  cp.srcsum[n] = ssum;
}

// ---------------------------------------------------------------------------
// Deterministic health/conservation reduction: per block, the zeroth moment of
// every lattice, the first moment of the momentum lattice, the minimum
// population and the count of non-finite values.  partials: [block][L + D + 2]
// ---------------------------------------------------------------------------
// Block reductions of a 256-thread block: a butterfly over the 64 lanes of each
// wave (cross-lane moves, no LDS), then the four wave results in wave order.  The
// order is fixed, so a reduction gives the same bits on every call.  The result is
// valid in thread 0; sh holds 4 doubles and is free again on return.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  v = wave_sum(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_min(double v, double *sh) {
  const int t = threadIdx.x;
  v = wave_min(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  const double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  return r;
}

// Internal energy of the adsorbed phase before this step's chemistry, at this
// step's temperature (eq temperatureCell, adsorbed part).
__global__ __launch_bounds__(256) void k_surface_energy(const KParams p) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= p.N) return;
  const double T = p.T_cur[n];
  double es = 0.0;
  for (int k = 0; k < p.K; ++k) es += p.theta[(size_t)k * p.N + n] * (p.es_u[k] + p.es_c[k] * T);
  p.rEs[n] = es;
}

// Totals of the stored state.  Species populations include the reaction
// population the last step added after its collision (p.src_prev).  Every thread
// forms its node's W = L + D + 2 values first (lattice masses, momentum-lattice
// momentum, minimum population, non-finite count); the block then reduces all of
// them at once, each by the same tree (wave butterfly, then the four waves in a
// fixed order), with one barrier.
template <int D, int L, typename PT>
__global__ __launch_bounds__(256) void k_diag(int Mmom, const KParams p, const PT *pop, double *partials) {
  constexpr int Q = LQ<D>::Q, W = L + D + 2;
  __shared__ double sh[W][4];
  const int N = p.N;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = threadIdx.x;
  double val[W];
  double mn = INFINITY, bad = 0.0;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    double s = 0.0;
    if (n < N) {
      const bool src = l < p.M && p.src_prev;
      const double km = src ? p.theta_ref * p.mmin_over_m[l < LBM_MMAX ? l : 0] : 0.0;
      const double *sa = p.rec_prev + (size_t)(kRecSrc + (l < LBM_MMAX ? l : 0)) * N;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        double v = (double)pop[(size_t)(l * Q + i) * N + n];
        if (src) v += source_population<D>(load_src<D>(p.rec_prev, sa, p.T_prev, (size_t)N, n), km, p.inv_T_ref, i);
        if (!isfinite(v)) bad += 1.0;
        s += v;
        mn = fmin(mn, v);
      }
    }
    val[l] = s;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double s = 0.0;
    if (n < N) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c = ((d == 0 ? i : (d == 1 ? i / 3 : i / 9)) % 3) - 1;
        s += c * (double)pop[(size_t)(Mmom * Q + i) * N + n];
      }
    }
    val[L + d] = s;
  }
  val[L + D] = mn;
  val[L + D + 1] = bad;
#pragma unroll
  for (int k = 0; k < W; ++k) val[k] = (k == L + D) ? wave_min(val[k]) : wave_sum(val[k]);
  if ((t & 63) == 0) {
#pragma unroll
    for (int k = 0; k < W; ++k) sh[k][t >> 6] = val[k];
  }
  __syncthreads();
  if (t < W) {
    const double r = (t == L + D) ? fmin(fmin(sh[t][0], sh[t][1]), fmin(sh[t][2], sh[t][3]))
                                  : (sh[t][0] + sh[t][1]) + (sh[t][2] + sh[t][3]);
    partials[(size_t)blockIdx.x * W + t] = r;
  }
}

// Totals of the per-block partials [nblocks][W]: thread w adds column w over the
// blocks in block order (the minimum for column W - 2), the order a host loop over
// the partials takes, so the totals equal such a loop's bit for bit.
__global__ __launch_bounds__(64) void k_diag_totals(const double *partials, int nblocks, int W, double *totals) {
  const int w = threadIdx.x;
  if (w >= W) return;
  const bool is_min = w == W - 2;
  double acc = is_min ? INFINITY : 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double v = partials[(size_t)b * W + w];
    acc = is_min ? fmin(acc, v) : acc + v;
  }
  totals[w] = acc;
}

// Tiles of 64 nodes per species block.  A D3Q27 block of M + 1 waves takes 78 KB of LDS
// and about 156 VGPRs: two such blocks would fit a CU's 160 KB of LDS and 512 registers
// per lane, but the waves of a block are placed from the first SIMD on, so two 6-wave
// blocks would need four waves on one SIMD and only one block runs per CU.  One block
// of two tiles (12 waves, three per SIMD) puts both on the CU; each tile keeps its own
// barriers (tile_sync).
template <int D, int M>
constexpr int kSpeciesTiles = (D == 3 && M == 5) ? 2 : 1;

unsigned padded_blocks(int N, int bs) {
  unsigned nb = (unsigned)((N + bs - 1) / bs);
  return (nb + 7u) & ~7u;
}

template <int D, int M, typename PT>
hipError_t species_dispatch_p(const KParams &p, hipStream_t s) {
  if constexpr (D == 1) {
    if (!p.energy) {                                  // one node per lane
      hipLaunchKernelGGL((k_species_lane<M, PT>), dim3(padded_blocks(p.N, 256)), dim3(256), 0, s, p);
      return hipGetLastError();
    }
  }
  // XCD y slabs (see k_species) on 3-D grids whose rows hold whole blocks; the grid
  // then has exactly 8 k blocks and every block lies inside the grid
  auto slabs = [&](int tb) { return (D == 3 && !p.colflag && p.ny % 8 == 0 && p.nx % (64 * tb) == 0) ? 1 : 0; };
  KParams q = p;
  if (p.energy) {
    q.xcd_slabs = slabs(1);
    hipLaunchKernelGGL((k_species<D, M, true, PT, 1>), dim3(padded_blocks(p.N, 64)), dim3(64 * (M + 2)), 0, s, q);
  } else {
    constexpr int TB = kSpeciesTiles<D, M>;
    q.xcd_slabs = slabs(TB);
    hipLaunchKernelGGL((k_species<D, M, false, PT, TB>), dim3(padded_blocks(p.N, 64 * TB)), dim3(64 * TB * (M + 1)),
                       0, s, q);
  }
  return hipGetLastError();
}

template <int D, int M>
hipError_t species_dispatch_e(const KParams &p, hipStream_t s) {
  return p.fp32 ? species_dispatch_p<D, M, float>(p, s) : species_dispatch_p<D, M, double>(p, s);
}

template <int D, int M, typename PT>
hipError_t mixture_dispatch_p(const KParams &p, hipStream_t s) {
  const unsigned nb = padded_blocks(p.N, 256);
  if (p.energy)
    hipLaunchKernelGGL((k_mixture<D, M, true, PT>), dim3(nb), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_mixture<D, M, false, PT>), dim3(nb), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int D, int M>
hipError_t mixture_dispatch_e(const KParams &p, hipStream_t s) {
  return p.fp32 ? mixture_dispatch_p<D, M, float>(p, s) : mixture_dispatch_p<D, M, double>(p, s);
}

template <int D, int M, typename PT>
hipError_t moments_dispatch_p(const KParams &p, double *out, hipStream_t s) {
  const unsigned nb = padded_blocks(p.N, 256);
  if (p.energy)
    hipLaunchKernelGGL((k_moments<D, M, true, PT>), dim3(nb), dim3(256), 0, s, p, out);
  else
    hipLaunchKernelGGL((k_moments<D, M, false, PT>), dim3(nb), dim3(256), 0, s, p, out);
  return hipGetLastError();
}

template <int D, int M>
hipError_t moments_dispatch_e(const KParams &p, double *out, hipStream_t s) {
  return p.fp32 ? moments_dispatch_p<D, M, float>(p, out, s) : moments_dispatch_p<D, M, double>(p, out, s);
}

template <int D>
hipError_t species_dispatch(const KParams &p, hipStream_t s) {
  switch (p.M) {
    case 2: return species_dispatch_e<D, 2>(p, s);
    case 3: return species_dispatch_e<D, 3>(p, s);
    case 4: return species_dispatch_e<D, 4>(p, s);
    case 5: return species_dispatch_e<D, 5>(p, s);
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t mixture_dispatch(const KParams &p, hipStream_t s) {
  switch (p.M) {
    case 2: return mixture_dispatch_e<D, 2>(p, s);
    case 3: return mixture_dispatch_e<D, 3>(p, s);
    case 4: return mixture_dispatch_e<D, 4>(p, s);
    case 5: return mixture_dispatch_e<D, 5>(p, s);
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t moments_dispatch(const KParams &p, double *out, hipStream_t s) {
  switch (p.M) {
    case 2: return moments_dispatch_e<D, 2>(p, out, s);
    case 3: return moments_dispatch_e<D, 3>(p, out, s);
    case 4: return moments_dispatch_e<D, 4>(p, out, s);
    case 5: return moments_dispatch_e<D, 5>(p, out, s);
  }
  return hipErrorInvalidValue;
}

template <int D, typename PT>
hipError_t init_dispatch_p(const InitParams &ip, hipStream_t s) {
  const unsigned nb = (unsigned)((ip.N + 255) / 256);
  switch (ip.M) {
    case 2: hipLaunchKernelGGL((k_init<D, 2, PT>), dim3(nb), dim3(256), 0, s, ip); break;
    case 3: hipLaunchKernelGGL((k_init<D, 3, PT>), dim3(nb), dim3(256), 0, s, ip); break;
    case 4: hipLaunchKernelGGL((k_init<D, 4, PT>), dim3(nb), dim3(256), 0, s, ip); break;
    case 5: hipLaunchKernelGGL((k_init<D, 5, PT>), dim3(nb), dim3(256), 0, s, ip); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int D>
hipError_t init_dispatch(const InitParams &ip, hipStream_t s) {
  return ip.fp32 ? init_dispatch_p<D, float>(ip, s) : init_dispatch_p<D, double>(ip, s);
}

}  // namespace

hipError_t launch_init(int dim, const InitParams &ip, hipStream_t s) {
  switch (dim) {
    case 1: return init_dispatch<1>(ip, s);
    case 2: return init_dispatch<2>(ip, s);
    case 3: return init_dispatch<3>(ip, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_species(int dim, const KParams &p, hipStream_t s) {
  switch (dim) {
    case 1: return species_dispatch<1>(p, s);
    case 2: return species_dispatch<2>(p, s);
    case 3: return species_dispatch<3>(p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mixture(int dim, const KParams &p, hipStream_t s) {
  switch (dim) {
    case 1: return mixture_dispatch<1>(p, s);
    case 2: return mixture_dispatch<2>(p, s);
    case 3: return mixture_dispatch<3>(p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_moments(int dim, const KParams &p, double *out, hipStream_t s) {
  switch (dim) {
    case 1: return moments_dispatch<1>(p, out, s);
    case 2: return moments_dispatch<2>(p, out, s);
    case 3: return moments_dispatch<3>(p, out, s);
  }
  return hipErrorInvalidValue;
}

int chem_supported(int M, int K) {
  return (M == 2 && K == 2) || (M == 5 && K == 10) || (M == 3 && K == 4);
}

hipError_t launch_surface_energy(const KParams &p, hipStream_t s) {
  hipLaunchKernelGGL(k_surface_energy, dim3((p.N + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Current control (secant on each line's electrode potential): k_secant_start takes the
// line's present potential as the first iterate; k_secant reads the trial's end current
// I^(a) - target and forms the next iterate (stage 0: 10 mV above the first; stage 1: the
// secant update, none where the two last currents are equal), then fills the trial (or,
// for the final iterate, the step's) electrode potential of the line's nodes.
// One block per line: every thread forms the line's iterate (the same arithmetic), thread
// 0 stores the state once all have read it, and the block fills the line's nodes.
__global__ __launch_bounds__(256) void k_secant_start(const SecantParams s) {
  const int l = blockIdx.x;
  const double p = s.phi_line[l];
  if (threadIdx.x == 0) s.p0[l] = p;
  for (int n = s.off[l] + (int)threadIdx.x; n < s.off[l + 1]; n += 256) s.ped_try[n] = p;
}

__device__ __forceinline__ void secant_line(const SecantParams &s, int l, double ia_end) {
  const int b = s.off[l], e = s.off[l + 1];
  const double f = ia_end - s.target[l];
  const double p0 = s.p0[l], p1 = s.p1[l], f0 = s.f0[l];
  double p;
  if (s.stage == 0) {
    p = p0 + 0.01;
  } else {
    const double d = f - f0;
    p = d != 0.0 ? p1 - f * (p1 - p0) / d : p1;
  }
  __syncthreads();                              // every thread has read the state
  if (threadIdx.x == 0) {
    if (s.stage != 0) s.p0[l] = p1;
    s.f0[l] = f;
    s.p1[l] = p;
    if (s.final_iter) s.phi_line[l] = p;
  }
  double *dst = s.final_iter ? s.ped : s.ped_try;
  for (int n = b + (int)threadIdx.x; n < e; n += 256) dst[n] = p;
}

// Inclusive sum over the 256 threads of a block: each wave scans with lane shifts
// (no barrier), the four wave totals meet in LDS; every thread also receives the
// block total.
__device__ __forceinline__ double block_scan256(double v, double *s, double &total) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  __syncthreads();                              // earlier readers of s are done
  if (lane == 63) s[wv] = v;
  __syncthreads();
  double before = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k < wv) before += s[k];
  total = ((s[0] + s[1]) + s[2]) + s[3];
  return before + v;
}

// eqs areaCurrentDensity and electrolytePotential: one block per line, I^(a) and
// Phi_electrolyte as prefix sums along x from the line's first node (Phi = 0 before
// it), 256 cells at a time with the running totals carried.
// SEC: a trial of the current control; the block then also takes the line's secant
// step (k_secant below, fused so the trial costs one launch fewer).
template <bool SEC>
__global__ __launch_bounds__(256) void k_charge(const ChargeParams q, const SecantParams sp) {
  __shared__ double s[256];
  const int line = blockIdx.x;
  const int b = q.off[line], e = q.off[line + 1];
  double cia = 0.0, cpel = 0.0;                 // totals of the cells before this chunk
  int n = b + (int)threadIdx.x;
  double ivn = n < e ? q.iv[n] : 0.0, omn = n < e ? q.omega[n] : 0.0;
  for (int c0 = b; c0 < e; c0 += 256, n += 256) {
    const bool in = n < e;
    const double ivc = ivn, omc = omn;
    ivn = n + 256 < e ? q.iv[n + 256] : 0.0;    // the next chunk's loads cross this chunk's barriers
    omn = n + 256 < e ? q.omega[n + 256] : 0.0;
    double tot;
    const double ia = cia + block_scan256(in ? ivc * q.dx : 0.0, s, tot);
    cia += tot;
    const double pel = cpel + block_scan256(in ? ia * omc * q.dx : 0.0, s, tot);
    cpel += tot;
    if (in) {
      q.ia[n] = ia;
      q.pel[n] = pel;
    }
  }
  if constexpr (SEC) secant_line(sp, line, cia);    // cia: I^(a) at the line's last node
}

hipError_t launch_secant_start(const SecantParams &sp, hipStream_t s) {
  hipLaunchKernelGGL(k_secant_start, dim3(sp.lines), dim3(256), 0, s, sp);
  return hipGetLastError();
}

hipError_t launch_charge(const ChargeParams &q, const SecantParams *sp, hipStream_t s) {
  if (sp)
    hipLaunchKernelGGL(k_charge<true>, dim3(q.lines), dim3(256), 0, s, q, *sp);
  else
    hipLaunchKernelGGL(k_charge<false>, dim3(q.lines), dim3(256), 0, s, q, SecantParams{});
  return hipGetLastError();
}

hipError_t launch_chem(const ChemParams &cp, hipStream_t s) {
  if (cp.K == 0) {
    const unsigned nb = (unsigned)((cp.N + 255) / 256);
    switch (cp.M) {
      case 2: hipLaunchKernelGGL((k_faradaic<2>), dim3(nb), dim3(256), 0, s, cp); break;
      case 3: hipLaunchKernelGGL((k_faradaic<3>), dim3(nb), dim3(256), 0, s, cp); break;
      case 4: hipLaunchKernelGGL((k_faradaic<4>), dim3(nb), dim3(256), 0, s, cp); break;
      case 5: hipLaunchKernelGGL((k_faradaic<5>), dim3(nb), dim3(256), 0, s, cp); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const unsigned nb = (unsigned)((cp.N + 63) / 64);
  const dim3 bs(64);
  if (cp.M == 2 && cp.K == 2)
    hipLaunchKernelGGL((k_chem<2, 2>), dim3(nb), bs, 0, s, cp);
  else if (cp.M == 3 && cp.K == 4)
    hipLaunchKernelGGL((k_chem<3, 4>), dim3(nb), bs, 0, s, cp);
  else if (cp.M == 5 && cp.K == 10)
    hipLaunchKernelGGL((k_chem<5, 10>), dim3(nb), bs, 0, s, cp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int D, typename PT>
void diag_launch_l(int L, int Mmom, const KParams &p, const PT *q, double *partials, int nblocks, hipStream_t s) {
  switch (L) {       // lattices: M species + momentum (+ energy), M = 1..LBM_MMAX
    case 2: hipLaunchKernelGGL((k_diag<D, 2, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
    case 3: hipLaunchKernelGGL((k_diag<D, 3, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
    case 4: hipLaunchKernelGGL((k_diag<D, 4, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
    case 5: hipLaunchKernelGGL((k_diag<D, 5, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
    case 6: hipLaunchKernelGGL((k_diag<D, 6, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
    default: hipLaunchKernelGGL((k_diag<D, 7, PT>), dim3(nblocks), dim3(256), 0, s, Mmom, p, q, partials); break;
  }
}

template <typename PT>
hipError_t diag_dispatch(int dim, int L, int Mmom, const KParams &p, const void *pop, double *partials,
                         int nblocks, hipStream_t s) {
  const PT *q = static_cast<const PT *>(pop);
  if (L < 2 || L > LBM_MMAX + 2) return hipErrorInvalidValue;
  switch (dim) {
    case 1: diag_launch_l<1, PT>(L, Mmom, p, q, partials, nblocks, s); break;
    case 2: diag_launch_l<2, PT>(L, Mmom, p, q, partials, nblocks, s); break;
    default: diag_launch_l<3, PT>(L, Mmom, p, q, partials, nblocks, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_diag_totals(const double *partials, int nblocks, int W, double *totals, hipStream_t s) {
  if (W > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag_totals, dim3(1), dim3(64), 0, s, partials, nblocks, W, totals);
  return hipGetLastError();
}

hipError_t launch_diag(int dim, int L, int Mmom, const KParams &p, const void *pop, double *partials,
                       int nblocks, hipStream_t s) {
  return p.fp32 ? diag_dispatch<float>(dim, L, Mmom, p, pop, partials, nblocks, s)
                : diag_dispatch<double>(dim, L, Mmom, p, pop, partials, nblocks, s);
}
