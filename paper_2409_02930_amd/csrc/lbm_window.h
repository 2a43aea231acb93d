// lbm_window.h -- fused multi-step kernel for one-dimensional lattices (D1Q3):
// species lattices, momentum lattice and surface chemistry of LBM_STEPS whole
// steps in one launch, with the node state held in registers in between.
//
// Device code only.  It is not compiled with the library: the library prepends
// a generated preamble (constants of the context written in as literals, and
// the mechanism's chemistry as the device functions chem_rates / chem_node)
// and compiles the whole for gfx950 with hiprtc (chem_jit.hip).
//
// Layout of the work.  Each wave owns a window of 64 consecutive nodes of the
// 1-D domain (one node per lane; packed columns are one domain with column
// ends marked in colflag).  A step at a node needs the state of the previous
// step within two nodes: the pull reads the neighbours' post-collision
// populations (and reaction populations), and the momentum lattice's
// Galilean-correction stencil reads the neighbours' rho u (1 - 3RT) - rho u^3 /
// phi^2, which come from their own pulls.  The neighbours' values are read from
// the adjacent lanes with wave shuffles, so after s steps the lanes within 2 s
// of a window edge hold stale values.  Windows therefore overlap: a window
// starts 2 LBM_STEPS nodes before the nodes it owns and ends 2 LBM_STEPS nodes
// after them, and a wave stores only its inner 64 - 4 LBM_STEPS nodes.  Inlet,
// bounce-back and outflow ends read no neighbour, so a window may span several
// packed columns.  Nothing is exchanged between waves during a launch.
//
// Every step is the arithmetic of the species kernel (pull with the reaction
// populations of the previous step and the inlet equilibria, moments, node
// state, relaxation rates, species-momentum solve, Knudsen force, species
// collision; Sections 2.1-2.3, eqs density1, momentum1, tauab, betaa, tauak,
// transform1, netKnudsenForce, 27eq, 27qeq, fKnudsen, fStar,
// finalNumericalEquationsReactive), of the chemistry kernel (Section 4, eqs
// totalSurfaceReactionRate, rho_pc) and of the mixture kernel (eqs feqmix, Pex,
// f_source), written per node in the same order of operations.  Lanes that are
// already stale skip the chemistry.
//
// Preamble symbols: LBM_M, LBM_K, LBM_R, LBM_CHEM, LBM_FARADAIC, LBM_KNUDSEN,
// LBM_NEED_V, LBM_BC_LO, LBM_BC_HI (boundary kinds of the x ends),
// LBM_STEPS (odd), LBM_WPB (waves per block), KRECSRC, and the constants
// kThetaRef, kInvTRef, kNu, kMminOverM[M], kInvM[M], kImD[M][M],
// kInRho[2], kInRT[2], kInRhoA[2][M], kInRaT[2][M] (inlet states of the two ends).

#define LBM_WQ 3
#define LBM_WL (LBM_M + 1)
#define LBM_HALO (2 * LBM_STEPS)
#define LBM_USE (64 - 2 * LBM_HALO)
#define LBM_PERIODIC 0
#define LBM_BOUNCEBACK 1
#define LBM_INLET 2

#include "lbm_window_args.h"

// velocity of direction i (0, 1, 2 -> -1, 0, +1)
__device__ constexpr int lw_c(int i) { return i - 1; }
// lattice weight of direction i
__device__ constexpr double lw_w(int i) { return i == 1 ? (2.0 / 3.0) : (1.0 / 6.0); }

// Section 2.2: Psi_0 = 1 - P, Psi_{+1} = (xi + P)/2, Psi_{-1} = (-xi + P)/2
__device__ __forceinline__ double lw_psi(int c, double xi, double P) {
  return c == 0 ? (1.0 - P) : (c > 0 ? 0.5 * (xi + P) : 0.5 * (-xi + P));
}

// Reaction population the node adds to direction i of species lattice a
// (eq fsourceHetero): rho_dot_a dt Psi_i(v, v^2 + R_a T), all at this node.
__device__ __forceinline__ double lw_source(double sa, double T, double v, double km, int i) {
  const double RaT = km * (T * kInvTRef);
  double psi = sa;
  const double P = v * v + RaT;
  const int c = lw_c(i);
  psi *= (c == 0) ? 1.0 - P : 0.5 * (c * v + P);
  return psi;
}

// The separate kernels hand these values between waves or kernels through LDS or
// global memory, where the compiler cannot see how they were formed; hiding them
// here the same way keeps its choice of which product to fuse into an add the
// same, and so the rounding.
__device__ __forceinline__ double lw_opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Equilibrium entering direction i of lattice l through the inlet of end e
// (eq 27eq for a species, eq feqmix for the momentum lattice) at velocity vb.
__device__ __forceinline__ double lw_inlet(int e, int l, int i, double phi, double vb) {
  if (l < LBM_M) {
    const double P = vb * vb + kInRaT[e][l];
    return phi * kInRhoA[e][l] * lw_psi(lw_c(i), vb, P);
  }
  const double P = kInRT[e] + vb * vb;
  return phi * kInRho[e] * lw_psi(lw_c(i), vb, P);
}

// Without chemistry the step fits two waves per SIMD (256 registers); the
// chemistry's Newton system takes the whole register file of one wave.
#if LBM_CHEM
#define LBM_WIN_OCC
#else
#define LBM_WIN_OCC __attribute__((amdgpu_waves_per_eu(2, 2)))
#endif

extern "C" __global__ void __launch_bounds__(64 * LBM_WPB) LBM_WIN_OCC lbm_window(const WinArgs a) {
  constexpr int M = LBM_M, L = LBM_WL, Q = LBM_WQ;
  const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gw = blockIdx.x * LBM_WPB + wib;
  const int N = a.N;
  const int n = gw * LBM_USE - LBM_HALO + lane;
  const bool valid = n >= 0 && n < N;
  const int nc = n < 0 ? 0 : (n >= N ? N - 1 : n);   // lanes outside the domain read node 0 or N-1
  // lanes outside the domain are isolated nodes: both ends closed, no neighbour read
  int flag = 3;
  if (valid) flag = a.colflag ? (int)a.colflag[nc] : ((nc == 0 ? 1 : 0) | (nc == a.nx - 1 ? 2 : 0));
  const bool lo_miss = (flag & 1) && LBM_BC_LO != LBM_PERIODIC;
  const bool hi_miss = (flag & 2) && LBM_BC_HI != LBM_PERIODIC;
  const bool inlet_node = (lo_miss && LBM_BC_LO == LBM_INLET) || (hi_miss && LBM_BC_HI == LBM_INLET);
  const size_t sN = (size_t)N;

  const double phi = a.phi[nc];
  const double T = a.Tf[nc];
  const double kf = LBM_KNUDSEN ? a.kfac[nc] : 1.0;
  double fp[L][Q];                       // post-collision populations of the last step
#pragma unroll
  for (int l = 0; l < L; ++l)
#pragma unroll
    for (int i = 0; i < Q; ++i) fp[l][i] = a.pin[(size_t)(l * Q + i) * sN + nc];
  double vprev = LBM_NEED_V ? a.rec_prev[nc] : 0.0;   // v = u / phi of the last step
  double sa[M];                          // reaction source rho_dot_a dt of the last step
#pragma unroll
  for (int s = 0; s < M; ++s) sa[s] = LBM_CHEM ? a.rec_prev[(size_t)(KRECSRC + s) * sN + nc] : 0.0;
#if LBM_CHEM
  double th[LBM_K];
#pragma unroll
  for (int k = 0; k < LBM_K; ++k) th[k] = a.theta_in[(size_t)k * sN + nc];
#if LBM_SK_LDS
  __shared__ double sk_l[LBM_WPB][2 * LBM_R][64];
  double *skw = &sk_l[wib][0][lane];
#else
  double *skw = a.skg + (size_t)gw * (2 * LBM_R) * 64 + lane;
#endif
  chem_rates(T, skw);                    // isothermal: the rate constants hold for the launch
  __shared__ double sy[LBM_WPB][LBM_M + LBM_K][64];
  const double far_rate = LBM_FARADAIC ? a.far[nc] : 0.0;
#endif
  double ssum = 0.0, rhom_last = 1.0, vnew = 0.0;
#if LBM_CHEM
  __shared__ double stash[LBM_WPB][LBM_M * LBM_WQ + 2 * LBM_WQ + 1][64];
#endif
#pragma unroll 1
  for (int step = 0; step < LBM_STEPS; ++step) {
    const int edge = lane < 63 - lane ? lane : 63 - lane;
    const bool exact = valid && edge >= 2 * (step + 1);   // still exact after this step
    const double vb = inlet_node ? vprev : 0.0;

    // ---- pull: what this node sends in direction i is its post-collision
    //      population plus its reaction population; the node takes direction +1
    //      from the lane below and -1 from the lane above, or at a closed end its
    //      own opposite (bounce-back) or same (inlet, outflow) direction
    double f[L][Q];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      double out[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) out[i] = fp[l][i];
      if (LBM_CHEM && l < M) {
        const double km = kMminOverM[l] * kThetaRef;
#pragma unroll
        for (int i = 0; i < Q; ++i) out[i] += lw_source(sa[l], T, vprev, km, i);
      }
      const double from_lo = __shfl_up(out[2], 1, 64);
      const double from_hi = __shfl_down(out[0], 1, 64);
      f[l][1] = out[1];
      f[l][2] = lo_miss ? (LBM_BC_LO == LBM_BOUNCEBACK ? out[0] : out[2]) : from_lo;
      f[l][0] = hi_miss ? (LBM_BC_HI == LBM_BOUNCEBACK ? out[2] : out[0]) : from_hi;
      if (inlet_node) {
        if (lo_miss && LBM_BC_LO == LBM_INLET) f[l][2] = lw_inlet(0, l, 2, phi, vb);
        if (hi_miss && LBM_BC_HI == LBM_INLET) f[l][0] = lw_inlet(1, l, 0, phi, vb);
      }
    }

    // ---- moments (eqs density1, momentum1, fdensity, f1momMomentum)
    double m0[L], m1[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        s0 += f[l][i];
        s1 += lw_c(i) * f[l][i];
      }
      m0[l] = lw_opaque(s0);
      m1[l] = lw_opaque(s1);
    }

    // ---- node state (Section 2.1; temperature held)
    const double iphi = 1.0 / phi;
    const double rho = m0[M] * iphi;
    const double irho = 1.0 / rho;
    const double u = m1[M] * irho;
    const double v = u * iphi;
    double rs = 0.0, rho_a[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
      rho_a[s] = m0[s] * iphi;
      rs += rho_a[s];
    }
    const double irs = 1.0 / rs;
    double Y[M], RaT[M], im = 0.0;
#pragma unroll
    for (int s = 0; s < M; ++s) {
      Y[s] = rho_a[s] * irs;
      im += Y[s] * kInvM[s];
    }
    double Ps = 0.0, RT = 0.0;
#pragma unroll
    for (int s = 0; s < M; ++s) {
      RaT[s] = kThetaRef * kMminOverM[s] * (T * kInvTRef);
      RT += Y[s] * RaT[s];
      Ps += rho_a[s] * RaT[s];
    }
    const double Tr = T * kInvTRef;
    const double g = Ps / (Tr * sqrt(Tr) * im);   // 1/tau_ab = R_a T g / (m_b D_ab^ref)

    // ---- relaxation rates and the species-momentum system (eqs tauab, betaa,
    //      tauak, transform1 with the Knudsen terms)
    double iab[M][M], beta[M], itk[M], A[M][M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const double rg = RaT[s] * g;
      double it = 0.0;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        iab[s][c] = (c != s) ? rg * kImD[s][c] : 0.0;
        it += Y[c] * iab[s][c];
      }
      beta[s] = it / (2.0 + it);
      itk[s] = LBM_KNUDSEN ? sqrt(RaT[s]) / kf : 0.0;
#pragma unroll
      for (int c = 0; c < M; ++c)
        A[s][c] = lw_opaque((c == s) ? 1.0 + 0.5 * it + 0.5 * itk[s] : -0.5 * Y[s] * iab[s][c]);
    }
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
    for (int s = 0; s < M; ++s) x[s] = m1[s];
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
    for (int s = 0; s < M; ++s) x[s] = lw_opaque(x[s]);
    double fk = 0.0;                            // eq netKnudsenForce
#pragma unroll
    for (int c = 0; c < M; ++c) fk -= x[c] * lw_opaque(itk[c]);
    const double rA = rho * u * (1.0 - 3.0 * RT) - rho * u * v * v;

    // ---- species collision
    double te[M][Q], ts[M][Q], dlt[M][Q];
#pragma unroll
    for (int s = 0; s < M; ++s) RaT[s] = lw_opaque(RaT[s]);   // selected per species wave in the kernel
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const double pra = m0[s];
      const bool pos = pra > 0.0;
      const double ipra = pos ? 1.0 / pra : 0.0;
      const double xs = x[s] * ipra;
      const double Pe = v * v + RaT[s], Pst = xs * xs + RaT[s];
      te[s][0] = 0.5 * (-v + Pe); te[s][1] = 1.0 - Pe; te[s][2] = 0.5 * (v + Pe);
      ts[s][0] = 0.5 * (-xs + Pst); ts[s][1] = 1.0 - Pst; ts[s][2] = 0.5 * (xs + Pst);
#pragma unroll
      for (int i = 0; i < Q; ++i) dlt[s][i] = lw_opaque(pra * (te[s][i] - ts[s][i]));
    }
    double fn[L][Q];
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const double pra = m0[s];
      const bool pos = pra > 0.0;
      double tk[Q];
      tk[0] = 0.5 * RaT[s]; tk[1] = 1.0 - RaT[s]; tk[2] = 0.5 * RaT[s];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        double F = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) F += iab[s][c] * dlt[c][i];
        const double feq = pra * te[s][i];
        const double fst = pos ? pra * ts[s][i] : 0.0;
        const double fkn = pra * tk[i];
        const double Fi = Y[s] * F + itk[s] * (fst - fkn);
        const double f0 = f[s][i];
        fn[s][i] = f0 + 2.0 * beta[s] * (feq - f0) + (beta[s] - 1.0) * Fi;
      }
    }

    const bool own = valid && lane >= LBM_HALO && lane < 64 - LBM_HALO;
    if (step == LBM_STEPS - 1 && own) {      // records of the launch's last step
      a.rRT[n] = RT;
      a.rA[n] = rA;
      if (LBM_KNUDSEN) a.rFk[n] = fk;
#if LBM_CHEM
#pragma unroll
      for (int s = 0; s < M; ++s) a.rrho[(size_t)s * sN + n] = rho_a[s];
#endif
    }

    // ---- momentum lattice: extended equilibrium with the Galilean correction
    //      from the neighbours' rA (mirror at closed ends) and the Knudsen force;
    //      the chemistry's mass source term is added once the chemistry has run
    double fmb[Q], fex[Q];
    {
      double sf = 0.0, jf = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        sf += f[M][i];
        jf += lw_c(i) * f[M][i];
      }
      const double rhom = sf / phi;
      const double um = jf / rhom;
      const double vm = um / phi;
      const double RTm = lw_opaque(RT), rAm = lw_opaque(rA), fkm = lw_opaque(fk);
      const double omega = 1.0 / (kNu / RTm + 0.5);
      const double rA_lo = __shfl_up(rAm, 1, 64);
      const double rA_hi = __shfl_down(rAm, 1, 64);
      constexpr bool nonper = LBM_BC_LO != LBM_PERIODIC;
      double G = 0.0;
      G += lw_w(0) * lw_c(0) * ((nonper && (flag & 1)) ? rAm : rA_lo);
      G += lw_w(2) * lw_c(2) * ((nonper && (flag & 2)) ? rAm : rA_hi);
      const double gfac = (2.0 - omega) / (2.0 * phi * rhom * omega);
      G *= 3.0;
      const double Pex = RTm + vm * vm + gfac * G;
      const double Fk = LBM_KNUDSEN ? fkm : 0.0;
      const double xi = (um + Fk / (omega * rhom)) / phi;
      const double phirho = phi * rhom;
      rhom_last = rhom;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        fex[i] = phirho * lw_psi(lw_c(i), xi, Pex);
        fmb[i] = f[M][i] + omega * (fex[i] - f[M][i]);
      }
    }

    // ---- surface chemistry of the node (stale lanes skip it); what the step
    //      still needs afterwards waits in LDS meanwhile
    double src[M];
#pragma unroll
    for (int s = 0; s < M; ++s) src[s] = 0.0;
    ssum = 0.0;
#if LBM_CHEM
    {
      double *st = &stash[wib][0][lane];
      int k = 0;
#pragma unroll
      for (int s = 0; s < M; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i) st[64 * k++] = fn[s][i];
#pragma unroll
      for (int i = 0; i < Q; ++i) { st[64 * k++] = fmb[i]; st[64 * k++] = fex[i]; }
      st[64 * k++] = v;
#pragma unroll
      for (int s = 0; s < M; ++s) rho_a[s] = lw_opaque(rho_a[s]);
      if (exact)
        chem_node(phi, rho_a, th, far_rate, LBM_FARADAIC, a.fuel, a.product, a.dt, a.rho_unit, skw, sy[wib], lane,
                  src, ssum);
      k = 0;
#pragma unroll
      for (int s = 0; s < M; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i) fn[s][i] = st[64 * k++];
#pragma unroll
      for (int i = 0; i < Q; ++i) { fmb[i] = st[64 * k++]; fex[i] = st[64 * k++]; }
      vnew = st[64 * k++];
    }
#else
    vnew = v;
#endif
    {
      const double ratio = LBM_CHEM ? lw_opaque(ssum) / (phi * rhom_last) : 0.0;   // rho_pc / rho - 1
#pragma unroll
      for (int i = 0; i < Q; ++i) fn[M][i] = fmb[i] + ratio * fex[i];
    }

#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int i = 0; i < Q; ++i) fp[l][i] = fn[l][i];
#pragma unroll
    for (int s = 0; s < M; ++s) sa[s] = lw_opaque(src[s]);   // node records of the step
    vprev = lw_opaque(vnew);
  }

  // ---- the window's own nodes: state after the last step
  if (valid && lane >= LBM_HALO && lane < 64 - LBM_HALO) {
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(fp[l][i], a.pout + (size_t)(l * Q + i) * sN + n);
    if (LBM_NEED_V) a.rec_out[n] = vprev;
#if LBM_CHEM
#pragma unroll
    for (int s = 0; s < M; ++s) a.rec_out[(size_t)(KRECSRC + s) * sN + n] = sa[s];
    a.srcsum[n] = ssum;
#pragma unroll
    for (int k = 0; k < LBM_K; ++k) a.theta_out[(size_t)k * sN + n] = th[k];
#endif
  }
}
