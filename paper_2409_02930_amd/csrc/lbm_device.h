// lbm_device.h -- device helpers shared by the forward and adjoint kernels:
// lattice directions and weights, the product-form Psi of Section 2.2, the
// energy equilibrium, node geometry and the pull-stream addressing with its
// boundary rules.  Header-only; every translation unit gets its own copy.
#ifndef LBM_DEVICE_H
#define LBM_DEVICE_H

#include "lbm_internal.h"

#include <math.h>

namespace {

template <int D> struct LQ { static constexpr int Q = (D == 1) ? 3 : (D == 2 ? 9 : 27); };

// velocity component a of direction i: i = sum_a (c_ia + 1) 3^a
__host__ __device__ constexpr int cdir(int i, int a) {
  return (a == 0 ? i : (a == 1 ? i / 3 : i / 9)) % 3 - 1;
}

template <int D> __host__ __device__ constexpr int cnorm2(int i) {
  return (cdir(i, 0) != 0) + (D > 1 ? (cdir(i, 1) != 0) : 0) + (D > 2 ? (cdir(i, 2) != 0) : 0);
}

// lattice weight: product form at xi = 0, P = 1/3
template <int D> __device__ constexpr double wdir(int i) {
  double w = 1.0;
  for (int a = 0; a < D; ++a) w *= (cdir(i, a) == 0) ? (2.0 / 3.0) : (1.0 / 6.0);
  return w;
}

// Section 2.2: Psi_0 = 1 - P, Psi_{+1} = (xi + P)/2, Psi_{-1} = (-xi + P)/2
__device__ __forceinline__ double psi1(int c, double xi, double P) {
  return c == 0 ? (1.0 - P) : (c > 0 ? 0.5 * (xi + P) : 0.5 * (-xi + P));
}

// product form Psi_i for one direction (i may be a run-time value)
template <int D>
__device__ __forceinline__ double psi_dir(int i, const double *xi, const double *P) {
  double r = psi1(cdir(i, 0), xi[0], P[0]);
  if (D > 1) r *= psi1(cdir(i, 1), xi[1], P[1]);
  if (D > 2) r *= psi1(cdir(i, 2), xi[2], P[2]);
  return r;
}

// Energy equilibrium (Section 3.3 with O_a = RT d/dv_a + v_a): per direction
//   a(c) = Psi_c(v, RT + v^2),
//   e(0) = v^2/2 - (RT^2 + 5/2 RT v^2 + v^4/2),
//   e(+-1) = (+-(RT v + v^3/2) + RT^2 + 5/2 RT v^2 + v^4/2) / 2,
//   g_i = phi rho [U prod_a a_a + sum_b e_b prod_{a != b} a_a].
template <int D>
__device__ __forceinline__ double geq_dir(int i, double phirho, double U, double RT, const double *v) {
  double av[3], ev[3];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int c = cdir(i, d);
    const double vd = v[d];
    const double P1 = RT + vd * vd;
    const double xiE = RT * vd + 0.5 * vd * vd * vd;
    const double PE = RT * RT + 2.5 * RT * vd * vd + 0.5 * vd * vd * vd * vd;
    av[d] = psi1(c, vd, P1);
    ev[d] = (c == 0) ? (0.5 * vd * vd - PE) : (c > 0 ? 0.5 * (xiE + PE) : 0.5 * (-xiE + PE));
  }
  double pa = av[0];
#pragma unroll
  for (int d = 1; d < D; ++d) pa *= av[d];
  double acc = U * pa;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    double t = ev[b];
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (d != b) t *= av[d];
    acc += t;
  }
  return phirho * acc;
}

struct Node {
  int n, x, y, z;
  int flag;   // bit0: x-low boundary node, bit1: x-high boundary node
};

// XCD-aware block order: hardware hands block b to XCD b % 8; give each XCD a
// contiguous range of the domain so neighbouring rows share that XCD's L2.
__device__ __forceinline__ bool get_node(const KParams &p, Node &nd) {
  const unsigned nb = gridDim.x;               // multiple of 8 (host pads)
  const unsigned per = nb >> 3;
  const unsigned b = blockIdx.x;
  const unsigned lb = (b & 7u) * per + (b >> 3);
  const int n = (int)(lb * blockDim.x + threadIdx.x);
  if (n >= p.N) return false;
  nd.n = n;
  if (p.colflag) {
    nd.x = nd.y = nd.z = 0;
    nd.flag = p.colflag[n];
  } else {
    nd.x = n % p.nx;
    const int r = n / p.nx;
    nd.y = r % p.ny;
    nd.z = r / p.ny;
    nd.flag = (nd.x == 0 ? 1 : 0) | (nd.x == p.nx - 1 ? 2 : 0);
  }
  return true;
}

// Inlet state of side kind-1 without indexing the argument block per lane.
struct InletSel {
  double rho, RT, U, rho_a, RaT;
};
__device__ __forceinline__ InletSel inlet_sel(const KParams &p, int kind, int lat) {
  const bool lo = kind == 1;
  InletSel r;
  r.rho = lo ? p.inlet[0].rho : p.inlet[1].rho;
  r.RT = lo ? p.inlet[0].RT : p.inlet[1].RT;
  r.U = lo ? p.inlet[0].U : p.inlet[1].U;
  r.rho_a = 0.0;
  r.RaT = 0.0;
#pragma unroll
  for (int a = 0; a < LBM_MMAX; ++a) {
    if (a == lat) {
      r.rho_a = lo ? p.inlet[0].rho_a[a] : p.inlet[1].rho_a[a];
      r.RaT = lo ? p.inlet[0].RaT[a] : p.inlet[1].RaT[a];
    }
  }
  return r;
}

// Source geometry of the pull at one node, computed once and shared by every
// lattice: the wrapped source coordinate along x for c_x = -1, 0, +1, the
// wrapped y-z row offset for every (c_y, c_z), and whether the node sits on a
// non-periodic x end.  Packed columns use x = n and a zero row offset; the
// first step (populations stored post-stream) uses zero shifts everywhere.
template <int D>
struct PullGeo {
  int xs[3];        // source x for c_x = -1, 0, +1 (index c_x + 1)
  int yz[3][3];     // nx * (y_src + ny * z_src) for (c_y + 1, c_z + 1)
  int xself;        // x of the node itself (outflow copy source)
  bool lo_wall, hi_wall;
};

template <int D>
__device__ __forceinline__ PullGeo<D> pull_geo(const KParams &p, const Node &nd) {
  PullGeo<D> g;
  const bool first = p.first_step != 0;
  g.lo_wall = !first && (nd.flag & 1) && p.bc_lo != BC_PERIODIC;
  g.hi_wall = !first && (nd.flag & 2) && p.bc_hi != BC_PERIODIC;
  const bool col = p.colflag != nullptr;
  const int x = col ? nd.n : nd.x;
  g.xself = x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = first ? 0 : k - 1;
    int xs = x - c;
    if (!col) { xs += (xs < 0) ? p.nx : 0; xs -= (xs >= p.nx) ? p.nx : 0; }
    g.xs[k] = xs;
  }
  int ys[3], zs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = first ? 0 : k - 1;
    ys[k] = nd.y;
    zs[k] = nd.z;
    if (D > 1) { ys[k] -= c; ys[k] += (ys[k] < 0) ? p.ny : 0; ys[k] -= (ys[k] >= p.ny) ? p.ny : 0; }
    if (D > 2) { zs[k] -= c; zs[k] += (zs[k] < 0) ? p.nz : 0; zs[k] -= (zs[k] >= p.nz) ? p.nz : 0; }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g.yz[a][b] = col ? 0 : p.nx * (ys[a] + p.ny * zs[b]);
  return g;
}

// Stored population that streams into direction i: returns the source node and
// sets the source direction.  Always an in-range address and free of branches:
// periodic wrap, bounce-back (own node, opposite direction) and outflow (copy
// of the same x, i.e. the zero-gradient extrapolation along x) are selects.
// Inlet directions read the node's own slot here and are replaced by the inlet
// equilibrium afterwards (inlet_kind).
template <int D>
__device__ __forceinline__ int pull_addr(const KParams &p, const Node &nd, const PullGeo<D> &g, int i,
                                         int &dir) {
  const int cx = cdir(i, 0);
  const int cy = D > 1 ? cdir(i, 1) : 0;
  const int cz = D > 2 ? cdir(i, 2) : 0;
  const bool miss = (cx == 1 && g.lo_wall) || (cx == -1 && g.hi_wall);
  const int kind = cx == 1 ? p.bc_lo : p.bc_hi;
  const int row = g.yz[cy + 1][cz + 1];
  dir = (miss && kind == BC_BOUNCEBACK) ? LQ<D>::Q - 1 - i : i;
  const int x = (miss && kind == BC_OUTFLOW) ? g.xself : g.xs[cx + 1];
  return (miss && kind != BC_OUTFLOW) ? nd.n : x + row;
}

// 1 or 2 when direction i of nd enters through the inlet at x-low or x-high.
template <int D>
__device__ __forceinline__ int inlet_kind(const KParams &p, const Node &nd, int i) {
  if (p.first_step) return 0;
  const int cx = cdir(i, 0);
  if (cx == 1 && (nd.flag & 1) && p.bc_lo == BC_INLET) return 1;
  if (cx == -1 && (nd.flag & 2) && p.bc_hi == BC_INLET) return 2;
  return 0;
}

// True when some direction of nd enters through an inlet.
__device__ __forceinline__ bool is_inlet_node(const KParams &p, const Node &nd) {
  return !p.first_step &&
         (((nd.flag & 1) && p.bc_lo == BC_INLET) || ((nd.flag & 2) && p.bc_hi == BC_INLET));
}

// Equilibrium population of lattice `lat` entering direction i of node n through
// the inlet of side kind (eq 27eq for species, eq feqmix for the momentum
// lattice, eq geq_i for the energy lattice) at the node velocity vb.  The
// energy lattice's inlet fixes the temperature of what enters: its equilibrium
// is that of the node's own mixture at the inlet temperature, from the records
// the previous step wrote for inlet nodes (density, U and R T, planes kRecEin..).
template <int D, int M>
__device__ __forceinline__ double inlet_population(const KParams &p, int kind, int lat, int i, int n,
                                                   double phi, const double *vb) {
  const InletSel in = inlet_sel(p, kind, lat);
  double P[D];
  if (lat < M) {
#pragma unroll
    for (int d = 0; d < D; ++d) P[d] = vb[d] * vb[d] + in.RaT;
    return phi * in.rho_a * psi_dir<D>(i, vb, P);
  }
  if (lat == M) {
#pragma unroll
    for (int d = 0; d < D; ++d) P[d] = in.RT + vb[d] * vb[d];
    return phi * in.rho * psi_dir<D>(i, vb, P);
  }
  const double *e = p.rec_prev + (size_t)kRecEin * p.N + n;
  return geq_dir<D>(i, phi * e[0], e[p.N], e[2 * (size_t)p.N], vb);
}

// Post-stream populations of lattice `lat` at node nd (pull scheme).  All Q
// loads are issued unconditionally; the inlet fix-up runs on inlet nodes only.
// Reaction population that the previous step added to species a in direction i
// at node y after its collision (eq fsourceHetero):
//   rho_dot_a dt prod_d Psi_{c_id}(v_d, v_d^2 + R_a T), all at node y.
// Adding it when the population is pulled, instead of writing it into the
// stored populations, saves a read-modify-write pass over every species
// population; the sum is the same.
//
// SrcVals: the record values of one source node: rho_dot_a dt, T, v.
template <int D>
struct SrcVals {
  double sa, T, v[D];
};

// rec: node records of the previous step (velocity planes first), sa: its
// source plane of species a, T: temperature of the previous step.
template <int D>
__device__ __forceinline__ SrcVals<D> load_src(const double *__restrict__ rec, const double *__restrict__ sa,
                                               const double *__restrict__ T, size_t N, int y) {
  SrcVals<D> r;
  r.sa = sa[y];
  r.T = T[y];
#pragma unroll
  for (int d = 0; d < D; ++d) r.v[d] = rec[d * N + y];
  return r;
}

// km = theta_ref m_min / m_a, so R_a T = km T / T_ref.
template <int D>
__device__ __forceinline__ double source_population(const SrcVals<D> &s, double km, double inv_T_ref, int i) {
  const double RaT = km * (s.T * inv_T_ref);
  double psi = s.sa;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double P = s.v[d] * s.v[d] + RaT;
    const int c = cdir(i, d);
    psi *= (c == 0) ? 1.0 - P : 0.5 * (c * s.v[d] + P);
  }
  return psi;
}

// Adds the reaction populations of species lattice a (source plane sa, km for
// a) to the pulled populations f, gathering every source node's record.
template <int D>
__device__ __forceinline__ void add_source_populations(const KParams &p, const Node &nd, const PullGeo<D> &g,
                                                       const double *sa, double km, double *f) {
  constexpr int Q = LQ<D>::Q;
  const size_t N = (size_t)p.N;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int dir;
    const int src = pull_addr<D>(p, nd, g, i, dir);
    f[i] += source_population<D>(load_src<D>(p.rec_prev, sa, p.T_prev, N, src), km, p.inv_T_ref, dir);
  }
}

// km = theta_ref m_min / m_lat without a run-time index into the parameters.
template <int M>
__device__ __forceinline__ double species_km(const KParams &p, int lat) {
  double km = 0.0;
#pragma unroll
  for (int c = 0; c < M; ++c) km += (c == lat ? 1.0 : 0.0) * p.mmin_over_m[c];
  return km * p.theta_ref;
}

// Raw pull of lattice lat: stored populations that stream into this node.
// Every stored population is read once, so the loads are non-temporal and
// leave the L2 to the node records that neighbouring nodes re-read.
// P: storage type of the populations (double, or float with double arithmetic).
template <int D, typename P = double>
__device__ __forceinline__ void pull_populations(const KParams &p, const Node &nd, const PullGeo<D> &g, int lat,
                                                 double *f) {
  constexpr int Q = LQ<D>::Q;
  const int N = p.N;
  const P *base = static_cast<const P *>(p.pin) + (size_t)lat * Q * N;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int dir;
    const int src = pull_addr<D>(p, nd, g, i, dir);
    f[i] = (double)__builtin_nontemporal_load(base + (size_t)dir * N + src);   // read once: keep L2 for records
  }
}

// Stores one population in storage type P (float: rounded to nearest).
template <typename P>
__device__ __forceinline__ void store_pop(void *out, size_t idx, double v) {
  __builtin_nontemporal_store((P)v, static_cast<P *>(out) + idx);
}

// Inlet directions of an inlet node take the inlet equilibrium.
template <int D, int M>
__device__ __forceinline__ void inlet_replace(const KParams &p, const Node &nd, int lat, double phi,
                                              const double *vb, double *f) {
  constexpr int Q = LQ<D>::Q;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int kind = inlet_kind<D>(p, nd, i);
    if (kind) f[i] = inlet_population<D, M>(p, kind, lat, i, nd.n, phi, vb);
  }
}

// Pulls lattice lat into f (post-stream populations of this node).  With SRC,
// species lattices also take the reaction population of the previous step at
// the source node and direction.
template <int D, int M, bool SRC = true, typename P = double>
__device__ __forceinline__ void pull_lattice(const KParams &p, const Node &nd, const PullGeo<D> &g,
                                             int lat, double phi, const double *vb, bool inlet_node,
                                             double *f) {
  pull_populations<D, P>(p, nd, g, lat, f);
  if (SRC && lat < M && p.src_prev)
    add_source_populations<D>(p, nd, g, p.rec_prev + (size_t)(kRecSrc + lat) * p.N, species_km<M>(p, lat), f);
  if (inlet_node) inlet_replace<D, M>(p, nd, lat, phi, vb, f);
}

// Node at x + c for the gradient stencil: periodic wrap, mirror ghost (the node
// itself) across non-periodic x ends.
template <int D>
__device__ __forceinline__ int nb_node(const KParams &p, const Node &nd, int i) {
  const int cx = cdir(i, 0);
  const int cy = D > 1 ? cdir(i, 1) : 0;
  const int cz = D > 2 ? cdir(i, 2) : 0;
  const bool nonper = p.bc_lo != BC_PERIODIC;
  if (nonper && ((cx == -1 && (nd.flag & 1)) || (cx == 1 && (nd.flag & 2)))) return nd.n;
  if (p.colflag) return nd.n + cx;
  int xs = nd.x + cx, ys = nd.y, zs = nd.z;
  xs += (xs < 0) ? p.nx : 0;
  xs -= (xs >= p.nx) ? p.nx : 0;
  if (D > 1) { ys += cy; ys += (ys < 0) ? p.ny : 0; ys -= (ys >= p.ny) ? p.ny : 0; }
  if (D > 2) { zs += cz; zs += (zs < 0) ? p.nz : 0; zs -= (zs >= p.nz) ? p.nz : 0; }
  return xs + p.nx * (ys + p.ny * zs);
}

}  // namespace

#endif  // LBM_DEVICE_H
