// Adjoint of K steps of the FP64 scheme with checkpoint-every-N recomputation.
//
// Forward record: the initial state, a checkpoint at every N-th step and the
// final state are kept; the wall force of states 1..K is written out.
// Backward: for each segment, newest first, the segment's states are rebuilt
// from its checkpoint and the steps are reversed one at a time.  A reversed
// step is three passes: moments of the stored state (the forward stencil
// input), the per-node vector-Jacobian product (transposed streaming and
// bounce-back gathered from the destinations, then the collision, forcing and
// equilibrium in reverse), and a gather that applies the transposed lattice
// gradient (with its wall ghosts) and the moment VJP.  The wall-force VJP is
// added at every recorded state.  The history of the initial state (forcing
// of f0) is reversed last.  Geometry adjoints are accumulated per node and
// finally carried through the reverse of the metric precompute (Christoffel
// symbols, inverse metric, determinant, metric products, both lattice
// stencils and the cubic continuation) to the chart and the wall displacement.
//
// The metric is static (no re-projection inside the K steps).  A wall may
// move with a fixed Cartesian velocity v: its chart components u_w = J^{-1} v
// at the wall row enter the bounce-back and the gradient ghost, and their
// dependence on J is carried back to the chart; v itself is a constant.
#include <type_traits>
#include <vector>

#include "lbm_adjoint.h"
#include "lbm_adjoint_node.h"

namespace lbm {

namespace {

__device__ __forceinline__ int wrapa(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

struct Node {
  int i, jf, k;
  unsigned n;  // fluid index (grids stay below 2^28 nodes)
};

// Element e of plane q of a [planes][N] array: a uniform plane base plus a
// 32-bit byte offset, so loads and stores keep the scalar-base form.
__device__ __forceinline__ const double& E(const double* __restrict__ a, long long q, const Grid& g, unsigned e) {
  return *(const double*)((const char*)(a + (size_t)q * g.N) + e * 8u);
}
__device__ __forceinline__ double& E(double* __restrict__ a, long long q, const Grid& g, unsigned e) {
  return *(double*)((char*)(a + (size_t)q * g.N) + e * 8u);
}

// Streaming (nontemporal) load and store of element e of plane q, for data a
// kernel touches once: they leave L2 to the planes that are read again.
__device__ __forceinline__ double EN(const double* __restrict__ a, long long q, const Grid& g, unsigned e) {
  return __builtin_nontemporal_load((const double*)((const char*)(a + (size_t)q * g.N) + e * 8u));
}
__device__ __forceinline__ void ESN(double* __restrict__ a, long long q, const Grid& g, unsigned e, double v) {
  __builtin_nontemporal_store(v, (double*)((char*)(a + (size_t)q * g.N) + e * 8u));
}
__device__ __forceinline__ bool fluid_node(const Grid& g, Node& p) {
  p.i = blockIdx.x * BX + threadIdx.x;
  p.jf = blockIdx.y * blockDim.y + threadIdx.y;
  p.k = blockIdx.z;
  if (p.i >= g.nx || p.jf >= g.H) return false;
  p.n = ((unsigned)p.k * g.H + p.jf) * g.nx + p.i;
  return true;
}

__device__ __forceinline__ unsigned nidx(const Grid& g, int i, int jf, int k) {
  return ((unsigned)k * g.H + jf) * g.nx + i;
}

// Row order of the node kernel (one 64-node row per workgroup): the hardware
// deals workgroups round-robin over the 8 XCDs, so the launch gives each XCD
// groups of ROW_GROUP consecutive rows in turn; a row's y-neighbours then sit
// in the same L2 (512x256x256: 10.19 -> 9.74 ms per launch).
constexpr int ROW_GROUP = 64;
inline unsigned row_group_blocks(const Grid& g) {
  const long long rows = (long long)((g.nx + BX - 1) / BX) * g.H * g.nz, per = 8LL * ROW_GROUP;
  return (unsigned)((rows + per - 1) / per * per);
}
__device__ __forceinline__ bool row_group_node(const Grid& g, Node& p) {
  const int ntx = (g.nx + BX - 1) / BX;
  const int xcd = (int)(blockIdx.x % 8), slot = (int)(blockIdx.x / 8);
  const int t = ((slot / ROW_GROUP) * 8 + xcd) * ROW_GROUP + slot % ROW_GROUP;
  if (t >= ntx * g.H * g.nz) return false;
  p.i = (t % ntx) * BX + threadIdx.x;
  p.jf = (t / ntx) % g.H;
  p.k = t / (ntx * g.H);
  if (p.i >= g.nx) return false;
  p.n = nidx(g, p.i, p.jf, p.k);
  return true;
}

// Full populations f(t) = w + pulled deviation + F(t-1)/2 of a stored state.
__device__ __forceinline__ void load_state(const Grid& g, const double* __restrict__ pop,
                                           const double* __restrict__ hist, const AGeo& G, const Node& p, double f[Q],
                                           double Fp[10]) {
#pragma unroll
  for (int q = 0; q < 10; ++q) Fp[q] = E(hist, q, g, p.n);
  double bp[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) bp[q] = Fp[4 + q];
  bp[0] -= Fp[0] / 3.0;
  bp[3] -= Fp[0] / 3.0;
  bp[5] -= Fp[0] / 3.0;
  const double isg = 1.0 / G.sg;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    double v;
    // plane l at the source node, or the bounce-back slot opp(l) here: one
    // uniform base (the lower plane), the choice is an offset
    constexpr int lo = l < opp(l) ? l : opp(l);
    const bool wall = (y > 0 && p.jf == 0) || (y < 0 && p.jf == g.H - 1);
    const unsigned es = nidx(g, wrapa(p.i - x, g.nx), p.jf - y, wrapa(p.k - z, g.nz));
    v = E(pop, lo, g, wall ? (unsigned)(opp(l) - lo) * (unsigned)g.N + p.n : (unsigned)(l - lo) * (unsigned)g.N + es);
    f[l] = wgt(l) + v + 0.5 * hermite_val<l>(isg, Fp[0], Fp + 1, bp);
  });
}

__device__ __forceinline__ void load_geo_full(const Grid& g, const double* __restrict__ geo, unsigned n, AGeo& G) {
  G.sg = 1.0 + E(geo, G_SG, g, n);
#pragma unroll
  for (int q = 0; q < 6; ++q) G.gi[q] = E(geo, (G_GI + q), g, n) + ((q == 0 || q == 3 || q == 5) ? 1.0 : 0.0);
#pragma unroll
  for (int q = 0; q < 18; ++q) G.gam[q] = E(geo, (G_GAM + q), g, n);
#pragma unroll
  for (int q = 0; q < 3; ++q) G.F[q] = E(geo, (G_F + q), g, n);
}

// Lattice gradient of the stored moments (ghost beyond a wall: -j_m, plus
// 2 rho u_w where the wall moves).
__device__ __forceinline__ void gradient_at(const Grid& g, const double* __restrict__ mom, const Node& p,
                                            const double* __restrict__ uw, int mv0, int mv1, double dj[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dj[a][b] = 0.0;
  // Branch-free: every neighbour's loads are issued unconditionally (the
  // solid neighbour's address is that of its ghost source), so that they
  // overlap instead of each waiting for its own round trip.
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    if (l == 0) return;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    const int in = wrapa(p.i + x, g.nx), kn = wrapa(p.k + z, g.nz), jn = p.jf + y;
    const bool fluid = y == 0 || (jn >= 0 && jn < g.H);
    const unsigned m = nidx(g, in, fluid ? jn : p.jf, kn);
    const double sgn = fluid ? 1.0 : -1.0;
    double jb[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) jb[b] = sgn * E(mom, (1 + b), g, m);
    if (y != 0 && (mv0 || mv1)) {
      // a moving wall's ghost is 2 rho u_w - j, with the column's u_w
      const int w = jn < 0 ? 0 : 1;
      const double rm = E(mom, 0, g, m);
      const double r2 = (!fluid && (w == 0 ? mv0 : mv1)) ? 2.0 * rm : 0.0;
      const size_t c = (((size_t)w * g.nz + kn) * g.nx + in) * 3;
#pragma unroll
      for (int b = 0; b < 3; ++b) jb[b] += r2 * uw[c + b];
    }
    constexpr double fct = 3.0 * wgt(l);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (x) dj[0][b] += (x * fct) * jb[b];
      if (y) dj[1][b] += (y * fct) * jb[b];
      if (z) dj[2][b] += (z * fct) * jb[b];
    }
  });
}

// a[q0 + q][n] += v[q] for q < NQ, every load before the first store (the
// planes of a may not be proven apart, so an interleaved read-modify-write
// would wait for each load in turn).
template <int NQ>
__device__ __forceinline__ void add_planes(double* __restrict__ a, int q0, const Grid& g, unsigned n, const double (&v)[NQ]) {
  double o[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) o[q] = E(a, q0 + q, g, n);
#pragma unroll
  for (int q = 0; q < NQ; ++q) E(a, q0 + q, g, n) = o[q] + v[q];
}

__device__ inline void add_geo_bar(const Grid& g, double* __restrict__ lg, unsigned n, const AGeoBar& gb) {
  double v[G_N];
  v[G_SG] = gb.sg;
#pragma unroll
  for (int q = 0; q < 6; ++q) v[G_GI + q] = gb.gi[q];
#pragma unroll
  for (int q = 0; q < 18; ++q) v[G_GAM + q] = gb.gam[q];
#pragma unroll
  for (int q = 0; q < 3; ++q) v[G_F + q] = gb.F[q];
  add_planes<G_N>(lg, 0, g, n, v);
}

__device__ inline void zero_bar(AGeoBar& gb) {
  gb.sg = 0;
  for (int q = 0; q < 6; ++q) gb.gi[q] = 0;
  for (int q = 0; q < 18; ++q) gb.gam[q] = 0;
  for (int q = 0; q < 3; ++q) gb.F[q] = 0;
}

// Moments rho, j of a stored state at every node.
__global__ __launch_bounds__(BX * BY) void k_adj_moments(Grid g, const double* __restrict__ pop, const double* __restrict__ hist,
                              const double* __restrict__ geo, double* __restrict__ mom) {
  Node p;
  if (!fluid_node(g, p)) return;
  AGeo G;
  load_geo_full(g, geo, p.n, G);
  double f[Q], Fp[10];
  load_state(g, pop, hist, G, p, f, Fp);
  double s = 0, j[3] = {0, 0, 0};
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    s += f[l];
    if (cx(l)) j[0] += cx(l) * f[l];
    if (cy(l)) j[1] += cy(l) * f[l];
    if (cz(l)) j[2] += cz(l) * f[l];
  });
  E(mom, 0, g, p.n) = G.sg * s;
  for (int a = 0; a < 3; ++a) E(mom, (1 + a), g, p.n) = G.sg * j[a];
}

// Adjoint s_l of f*_l at node p: f*_l(p) streamed to p + c_l, or bounced back
// into direction opp(l) at p across a wall.  lfn is the adjoint of the
// populations of the next state.
template <int l>
__device__ __forceinline__ double streamed_adjoint(const Grid& g, const double* __restrict__ lfn, const Node& p) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  constexpr int lo = l < opp(l) ? l : opp(l);
  const int jd = p.jf + y;
  const unsigned ed = nidx(g, wrapa(p.i + x, g.nx), jd, wrapa(p.k + z, g.nz));
  return E(lfn, lo, g,
           (jd >= 0 && jd < g.H) ? (unsigned)(l - lo) * (unsigned)g.N + ed : (unsigned)(opp(l) - lo) * (unsigned)g.N + p.n);
}
// The same, as a streaming load (the gather reads each value once).
template <int l>
__device__ __forceinline__ double streamed_adjoint_nt(const Grid& g, const double* __restrict__ lfn, const Node& p) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  constexpr int lo = l < opp(l) ? l : opp(l);
  const int jd = p.jf + y;
  const unsigned ed = nidx(g, wrapa(p.i + x, g.nx), jd, wrapa(p.k + z, g.nz));
  return EN(lfn, lo, g,
           (jd >= 0 && jd < g.H) ? (unsigned)(l - lo) * (unsigned)g.N + ed : (unsigned)(opp(l) - lo) * (unsigned)g.N + p.n);
}

// Reverse of one step at each node (mode 0), or of the history of an initial
// state (mode 1: only the new coefficients carry an adjoint).  The adjoints
// of the next state's populations enter through their Hermite basis sums; the
// direct adjoint of f is formed by the gather from lpb (the adjoint of the
// non-equilibrium flux P) and the same streamed adjoints.
// MW: some wall moves (walls at rest compile the moving-wall terms out).
template <bool MW>
__global__ __launch_bounds__(BX) void k_adj_node(Grid g, int mode, const double* __restrict__ pop, const double* __restrict__ hist,
                           const double* __restrict__ geo, const double* __restrict__ mom, double tau,
                           const double* __restrict__ lfn, const double* __restrict__ lpn, double* __restrict__ lpb,
                           double* __restrict__ lml, double* __restrict__ ldj, double* __restrict__ lpo,
                           double* __restrict__ lg, const double* __restrict__ uw, int mv0, int mv1,
                           double* __restrict__ ub, int fwall, const double* __restrict__ W,
                           const double* __restrict__ jac, double* __restrict__ lj) {
  Node p;
  if (!row_group_node(g, p)) return;
  const double th = 1.0 / 3.0;
  const bool with_old = mode == 0;
  // the geometry adjoint of the node is summed in LDS (one column of slots
  // per lane): it is added to from every stage of the reverse sweep
  __shared__ double gbs[G_N][BX];
#pragma unroll
  for (int q = 0; q < G_N; ++q) gbs[q][threadIdx.x] = 0.0;
  LdsGeoBar gb{&gbs[0][threadIdx.x], BX};
  // streaming loads and stores for what this kernel touches once (the
  // geometry, history, pulled populations and incoming coefficient adjoints;
  // the adjoints it hands on): L2 keeps the momentum and the next state's
  // adjoint, which neighbouring nodes read again
  AGeo G;
  G.sg = 1.0 + EN(geo, G_SG, g, p.n);
#pragma unroll
  for (int q = 0; q < 6; ++q) G.gi[q] = EN(geo, (G_GI + q), g, p.n) + ((q == 0 || q == 3 || q == 5) ? 1.0 : 0.0);
#pragma unroll
  for (int q = 0; q < 18; ++q) G.gam[q] = EN(geo, (G_GAM + q), g, p.n);
#pragma unroll
  for (int q = 0; q < 3; ++q) G.F[q] = EN(geo, (G_F + q), g, p.n);
  // forward: the moments of the state come from mom; the populations are
  // read once, for the non-equilibrium flux P, and not kept
  NodeFwd o;
  o.isg = 1.0 / G.sg;
  o.rho = E(mom, 0, g, p.n);
#pragma unroll
  for (int a = 0; a < 3; ++a) o.j[a] = E(mom, (1 + a), g, p.n);
  o.S0 = o.rho * o.isg;
#pragma unroll
  for (int a = 0; a < 3; ++a) o.S1[a] = o.j[a] * o.isg;
  {
    const double ir = 1.0 / o.rho;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b)
        o.a2[sym(a, b)] = o.rho * th * (G.gi[sym(a, b)] - (a == b ? 1.0 : 0.0)) + o.j[a] * o.j[b] * ir;
  }
  double Fp[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) Fp[q] = EN(hist, q, g, p.n);
#pragma unroll
  for (int q = 0; q < 6; ++q) o.bp[q] = Fp[4 + q];
  o.bp[0] -= th * Fp[0];
  o.bp[3] -= th * Fp[0];
  o.bp[5] -= th * Fp[0];
#pragma unroll
  for (int q = 0; q < 6; ++q) o.P[q] = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    constexpr int lo = l < opp(l) ? l : opp(l);
    const bool wall = (y > 0 && p.jf == 0) || (y < 0 && p.jf == g.H - 1);
    const unsigned es = nidx(g, wrapa(p.i - x, g.nx), p.jf - y, wrapa(p.k - z, g.nz));
    const double v = EN(pop, lo, g, wall ? (unsigned)(opp(l) - lo) * (unsigned)g.N + p.n : (unsigned)(l - lo) * (unsigned)g.N + es);
    const double ne = wgt(l) + v + 0.5 * hermite_val<l>(o.isg, Fp[0], Fp + 1, o.bp) - hermite_val<l>(o.isg, o.rho, o.j, o.a2);
    if (x) o.P[0] += ne;
    if (y) o.P[3] += ne;
    if (z) o.P[5] += ne;
    if (x && y) o.P[1] += (x * y) * ne;
    if (x && z) o.P[2] += (x * z) * ne;
    if (y && z) o.P[4] += (y * z) * ne;
  });
  // adjoint of the next state's populations, through their basis sums:
  // f*_l(x) went to x + c_l (or bounced back into direction opp(l) at x);
  // F_l(x)/2 was added to f_l(x, t+1)
  HSum hs, hb;
  hsum_zero(hs);
  hsum_zero(hb);
  if (with_old) {
    for_q([&](auto L) {
      constexpr int l = decltype(L)::value;
      hsum_add<l>(hs, streamed_adjoint<l>(g, lfn, p));
      hsum_add<l>(hb, 0.5 * E(lfn, l, g, p.n));
    });
    // the old forcing F(t-1) = H(Fp) is reversed first, so that Fp dies here
    HSum hFo;
    hFo.s0 = -0.5 * hs.s0;
#pragma unroll
    for (int a = 0; a < 3; ++a) hFo.s1[a] = -0.5 * hs.s1[a];
#pragma unroll
    for (int q = 0; q < 6; ++q) hFo.s2[q] = -0.5 * hs.s2[q];
    double Fpb[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) Fpb[q] = 0;
    double sgo = 0;
    old_forcing_vjp(hFo, o.isg, Fp, o.bp, Fpb, sgo);
    gb.add_sg(sgo);
#pragma unroll
    for (int q = 0; q < 10; ++q) ESN(lpo, q, g, p.n, Fpb[q]);
  }
  double dj[3][3];
  gradient_at(g, mom, p, uw, MW && mv0, MW && mv1, dj);
  node_fwd_rest(Fp, G, dj, tau, false, o);
  double cb[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) cb[q] = EN(lpn, q, g, p.n);
  double rb = 0, jb[3] = {0, 0, 0}, djb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Pb[6];
  // The wall force of this state, when the loss holds it (W = dL/dF of the
  // state, Sec. IV.A.2 traction sqrt g T^{iy} J): its adjoint of T joins the
  // step's in node_vjp, which is linear in it, and its adjoints of sqrt g and
  // J are added here, at the wall row only.
  double Tbf[6] = {0, 0, 0, 0, 0, 0};
  if (W && p.jf == (fwall == 0 ? 0 : g.H - 1)) {
    const double sgn = fwall == 0 ? -1.0 : 1.0;
    double J[3][3], ljv[9], sgb = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) J[a][b] = E(jac, (a * 3 + b), g, p.n);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double wj = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) wj += W[a] * J[a][i];
      Tbf[sym(i, 1)] += sgn * G.sg * wj;
      sgb += sgn * wj * o.T[sym(i, 1)];
#pragma unroll
      for (int a = 0; a < 3; ++a) ljv[a * 3 + i] = sgn * G.sg * W[a] * o.T[sym(i, 1)];
    }
    add_planes<9>(lj, 0, g, p.n, ljv);
    gb.add_sg(sgb);
  }
  node_vjp(nullptr, G, tau, with_old, o, hs, hb, cb, Tbf, Pb, rb, jb, djb, nullptr, gb);
  // moving walls: the bounce-back of a link into wall w loses
  // 6 (w_l / sqrt g) rho c_l . u_w (chart components u_w of the column)
  if (MW && with_old) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      if (!(w == 0 ? (p.jf == 0 && mv0) : (p.jf == g.H - 1 && mv1))) continue;
      const size_t c = (((size_t)w * g.nz + p.k) * g.nx + p.i) * 3;
      const double u[3] = {uw[c], uw[c + 1], uw[c + 2]};
      double isgb = 0, ubl[3] = {0, 0, 0};
      for_q([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr int y = cy(l);
        if ((w == 1 && y > 0) || (w == 0 && y < 0)) {
          const double cu = cx(l) * u[0] + y * u[1] + cz(l) * u[2];
          const double s = -6.0 * wgt(l) * streamed_adjoint<l>(g, lfn, p);
          rb += s * o.isg * cu;
          isgb += s * o.rho * cu;
          ubl[0] += s * o.isg * o.rho * cx(l);
          ubl[1] += s * o.isg * o.rho * y;
          ubl[2] += s * o.isg * o.rho * cz(l);
        }
      });
      gb.add_sg(-isgb * o.isg * o.isg);
#pragma unroll
      for (int a = 0; a < 3; ++a) ub[c + a] += ubl[a];
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) ESN(lpb, q, g, p.n, Pb[q]);
  ESN(lml, 0, g, p.n, rb);
#pragma unroll
  for (int a = 0; a < 3; ++a) ESN(lml, (1 + a), g, p.n, jb[a]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ESN(ldj, (a * 3 + b), g, p.n, djb[a][b]);
  // all 28 loads before the first store: the planes of lg may not be
  // proven apart, so an interleaved read-modify-write would wait for each
  // load in turn
  double lgv[G_N];
#pragma unroll
  for (int q = 0; q < G_N; ++q) lgv[q] = E(lg, q, g, p.n);
#pragma unroll
  for (int q = 0; q < G_N; ++q) E(lg, q, g, p.n) = lgv[q] + gbs[q][threadIdx.x];
}

// Transposed lattice gradient and the moment VJP:
// lf_out_l = (1 - 1/tau) s_l + pb_term_l(Pb) + sqrt g (rho_bar + j_bar . c_l)
// (+ lf_add_l), with s_l the streamed adjoint of the next state's populations
// lfn (none for the history of an initial state: lfn null) and
// j_bar = local + sum over the stencil of the neighbours' dj adjoints.
template <bool MW>
__global__ __launch_bounds__(BX * BY) void k_adj_gather(Grid g, const double* __restrict__ geo, const double* __restrict__ mom,
                             const double* __restrict__ lfn, double tau, const double* __restrict__ lpb,
                             const double* __restrict__ lml, const double* __restrict__ ldj,
                             const double* __restrict__ lf_add, double* __restrict__ lf_out, double* __restrict__ lg,
                             const double* __restrict__ uw, int mv0, int mv1, double* __restrict__ ub) {
  Node p;
  if (!fluid_node(g, p)) return;
  double rb = EN(lml, 0, g, p.n), jb[3] = {EN(lml, 1, g, p.n), EN(lml, 2, g, p.n), EN(lml, 3, g, p.n)};
  const double rho = EN(mom, 0, g, p.n);
  // the ghost of a moving wall, 2 rho u_w - j, also carries rho and u_w
  const bool mw0 = MW && p.jf == 0 && mv0, mw1 = MW && p.jf == g.H - 1 && mv1;
  const size_t c0 = ((size_t)p.k * g.nx + p.i) * 3, c1 = (((size_t)g.nz + p.k) * g.nx + p.i) * 3;
  double ub0[3] = {0, 0, 0}, ub1[3] = {0, 0, 0};
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    if (l == 0) return;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    constexpr double fct = 3.0 * wgt(l);
    // x_src = p - c_l used this node as its neighbour in direction l (no
    // branch: a solid x_src reads a fluid node of this layer and adds zero,
    // so the loads of all directions overlap)
    const int js = p.jf - y;
    {
      const bool fluid = y == 0 || (js >= 0 && js < g.H);
      const unsigned m = nidx(g, wrapa(p.i - x, g.nx), fluid ? js : p.jf, wrapa(p.k - z, g.nz));
      const double fm = fluid ? fct : 0.0;
      for (int b = 0; b < 3; ++b)
        jb[b] += fm * (x * E(ldj, (0 * 3 + b), g, m) + y * E(ldj, (1 * 3 + b), g, m) + z * E(ldj, (2 * 3 + b), g, m));
    }
    // wall ghost: node m' = p - (c_x, 0, c_z) in this layer, whose neighbour in
    // direction l is solid, used -j(p)
    if ((y < 0 && p.jf == 0) || (y > 0 && p.jf == g.H - 1)) {
      const unsigned m = nidx(g, wrapa(p.i - x, g.nx), p.jf, wrapa(p.k - z, g.nz));
      const bool mv = y < 0 ? mw0 : mw1;
      const size_t c = y < 0 ? c0 : c1;
      for (int b = 0; b < 3; ++b) {
        const double jgb =
            fct * (x * E(ldj, (0 * 3 + b), g, m) + y * E(ldj, (1 * 3 + b), g, m) + z * E(ldj, (2 * 3 + b), g, m));
        jb[b] -= jgb;
        if (mv) {
          rb += 2.0 * uw[c + b] * jgb;
          (y < 0 ? ub0 : ub1)[b] += 2.0 * rho * jgb;
        }
      }
    }
  });
  if (mw0)
    for (int b = 0; b < 3; ++b) ub[c0 + b] += ub0[b];
  if (mw1)
    for (int b = 0; b < 3; ++b) ub[c1 + b] += ub1[b];
  const double sg = 1.0 + EN(geo, G_SG, g, p.n);
  const double S0 = rho / sg, S1[3] = {EN(mom, 1, g, p.n) / sg, EN(mom, 2, g, p.n) / sg, EN(mom, 3, g, p.n) / sg};
  double Pb[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) Pb[q] = EN(lpb, q, g, p.n);
  const double keep = 1.0 - 1.0 / tau;
  double fb[Q];
  // the two optional inputs are tested once, outside the unrolled loop, so
  // that the loads of all directions are issued together
  auto fill = [&](auto has_s, auto has_a) {
    for_q([&](auto L) {
      constexpr int l = decltype(L)::value;
      double v = pb_term<l>(Pb);
      if constexpr (decltype(has_s)::value) v += keep * streamed_adjoint_nt<l>(g, lfn, p);
      if constexpr (decltype(has_a)::value) v += E(lf_add, l, g, p.n);
      fb[l] = v;
    });
  };
  using yes = std::true_type;
  using no = std::false_type;
  if (lfn) {
    if (lf_add)
      fill(yes{}, yes{});
    else
      fill(yes{}, no{});
  } else {
    if (lf_add)
      fill(no{}, yes{});
    else
      fill(no{}, no{});
  }
  double sgb = 0;
  moments_vjp(sg, S0, S1, rb, jb, fb, sgb);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    ESN(lf_out, l, g, p.n, fb[l]);
  });
  E(lg, G_SG, g, p.n) += sgb;
}

__device__ inline void inv3a(const double m[3][3], double r[3][3], double& det);

// The walls' chart-component velocity is u_w = J^{-1} v_w at the fluid node
// next to the wall: its adjoint ub passes to J there as -(J^{-T} ub) u_w^T.
__global__ __launch_bounds__(BX * BY) void k_adj_wall_velocity(Grid g, const double* __restrict__ jac,
                                                              const double* __restrict__ uw, int mv0, int mv1,
                                                              const double* __restrict__ ub, double* __restrict__ lj) {
  const int i = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  for (int w = 0; w < 2; ++w) {
    if (!(w == 0 ? mv0 : mv1)) continue;
    const unsigned n = nidx(g, i, w == 0 ? 0 : g.H - 1, k);
    const size_t c = (((size_t)w * g.nz + k) * g.nx + i) * 3;
    double J[3][3], Ji[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + n];
    double det;
    inv3a(J, Ji, det);
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) t[a] = Ji[0][a] * ub[c] + Ji[1][a] * ub[c + 1] + Ji[2][a] * ub[c + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) lj[(a * 3 + b) * g.N + n] -= t[a] * uw[c + b];
  }
}

// Wall-force VJP at one state: L += sum_a W_a F^a, F^a = sgn sum sqrt g
// T^{i y} J^a_i at the fluid layer next to `wall`.  Adds into lf (adjoint of
// f at this state), lg and lj.
__global__ __launch_bounds__(BX * BY) void k_adj_force(Grid g, int wall, const double* __restrict__ pop, const double* __restrict__ hist,
                            const double* __restrict__ geo, const double* __restrict__ jac, double tau,
                            const double* __restrict__ W, double* __restrict__ lf, double* __restrict__ lg,
                            double* __restrict__ lj) {
  Node p;
  p.i = blockIdx.x * BX + threadIdx.x;
  p.k = blockIdx.y * BY + threadIdx.y;
  if (p.i >= g.nx || p.k >= g.nz) return;
  p.jf = wall == 0 ? 0 : g.H - 1;
  p.n = nidx(g, p.i, p.jf, p.k);
  AGeo G;
  load_geo_full(g, geo, p.n, G);
  double f[Q], Fp[10];
  load_state(g, pop, hist, G, p, f, Fp);
  const double dj0[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  NodeFwd o;
  node_fwd(f, Fp, G, dj0, tau, false, o);
  const double sgn = wall == 0 ? -1.0 : 1.0;
  double J[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = E(jac, (a * 3 + b), g, p.n);
  // T^{i y} with y = 1: packed indices sym(i, 1)
  double Tb[6] = {0, 0, 0, 0, 0, 0};
  double sgb = 0, ljv[9];
  for (int i = 0; i < 3; ++i) {
    double wj = 0;
    for (int a = 0; a < 3; ++a) wj += W[a] * J[a][i];
    Tb[sym(i, 1)] += sgn * G.sg * wj;
    sgb += sgn * wj * o.T[sym(i, 1)];
    for (int a = 0; a < 3; ++a) ljv[a * 3 + i] = sgn * G.sg * W[a] * o.T[sym(i, 1)];
  }
  add_planes<9>(lj, 0, g, p.n, ljv);
  HSum h0;
  hsum_zero(h0);
  double cb[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double rb = 0, jb[3] = {0, 0, 0}, djb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Fpb[10], Pb[6];
  AGeoBar gb;
  zero_bar(gb);
  gb.sg = sgb;
  node_vjp(Fp, G, tau, false, o, h0, h0, cb, Tb, Pb, rb, jb, djb, Fpb, gb);
  double fb[Q];
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    fb[l] = pb_term<l>(Pb);
  });
  moments_vjp(G.sg, o.S0, o.S1, rb, jb, fb, gb.sg);
  add_planes<Q>(lf, 0, g, p.n, fb);
  add_geo_bar(g, lg, p.n, gb);
}

// ---------------------------------------------------- geometry adjoint
__device__ __forceinline__ long long eix(const Grid& g, int i, int j, int k) {
  return ((long long)k * (g.ny + 6) + (j + 3)) * g.nx + i;
}

__device__ inline void inv3a(const double m[3][3], double r[3][3], double& det) {
  det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
        m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
  const double id = 1.0 / det;
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) * id;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) * id;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) * id;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
}

// Fluid-node part: adjoints of Gamma, g^{-1}, det J and J^{-1} F back to
// D_l g (ldg), g (lge, packed) and J (lJe) on the extended grid.  g = J^T J
// at the node is formed from J, as the forward pass forms it.
__global__ __launch_bounds__(BX * BY) void k_adjg_fluid(Grid g, const double* __restrict__ wext,
                             const double* __restrict__ jac, double F0, double F1, double F2,
                             const double* __restrict__ lgv, const double* __restrict__ lj, double* __restrict__ ldg,
                             double* __restrict__ lge, double* __restrict__ lJe) {
  Node p;
  if (!fluid_node(g, p)) return;
  const int j = p.jf + 1;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const long long e = eix(g, p.i, j, p.k);
  double gm[3][3], gi[3][3], J[3][3], Ji[3][3], det, detJ;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + p.n];
  {
    double gq[6];
    metric_of(J, gq);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) gm[a][b] = gq[sym(a, b)];
  }
  inv3a(gm, gi, det);
  inv3a(J, Ji, detJ);
  double dg[3][6];
  for (int q = 0; q < 6; ++q) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int l = 1; l < Q; ++l) {
      const double fv = wext[q * NE + eix(g, wrapa(p.i + cx(l), g.nx), j + cy(l), wrapa(p.k + cz(l), g.nz))];
      s0 += wgt(l) * cx(l) * fv;
      s1 += wgt(l) * cy(l) * fv;
      s2 += wgt(l) * cz(l) * fv;
    }
    dg[0][q] = 3.0 * s0;
    dg[1][q] = 3.0 * s1;
    dg[2][q] = 3.0 * s2;
  }
  // Gamma^i_{jk} (packed jk) = 1/2 sum_l gi[i][l] (dg[j][kl] + dg[k][jl] - dg[l][jk])
  double gib[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // adjoint of the full matrix entries
  double dgb[3][6] = {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}};
  for (int ii = 0; ii < 3; ++ii)
    for (int jj = 0; jj < 3; ++jj)
      for (int kk = jj; kk < 3; ++kk) {
        const double lb = 0.5 * lgv[(G_GAM + ii * 6 + sym(jj, kk)) * g.N + p.n];
        for (int l = 0; l < 3; ++l) {
          gib[ii][l] += lb * (dg[jj][sym(kk, l)] + dg[kk][sym(jj, l)] - dg[l][sym(jj, kk)]);
          dgb[jj][sym(kk, l)] += lb * gi[ii][l];
          dgb[kk][sym(jj, l)] += lb * gi[ii][l];
          dgb[l][sym(jj, kk)] -= lb * gi[ii][l];
        }
      }
  // stored g^ij (packed, a <= b) used gi[a][b]
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const double v = lgv[(G_GI + sym(a, b)) * g.N + p.n];
      if (a == b)
        gib[a][a] += v;
      else {
        gib[a][b] += 0.5 * v;
        gib[b][a] += 0.5 * v;
      }
    }
  // gi = g^{-1}: gbar = -gi^T gib gi^T, then packed (off-diagonal counted twice)
  double t[3][3], gbf[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int c = 0; c < 3; ++c) s += gib[a][c] * gi[c][b];
      t[a][b] = s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int c = 0; c < 3; ++c) s += gi[c][a] * t[c][b];
      gbf[a][b] = -s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) lge[sym(a, b) * NE + e] = a == b ? gbf[a][a] : gbf[a][b] + gbf[b][a];
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 6; ++q) ldg[(l * 6 + q) * g.N + p.n] = dgb[l][q];
  // sqrt g = det J: d det / dJ = det J^{-T}
  double Jb[3][3];
  const double sgb = lgv[G_SG * g.N + p.n];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Jb[a][b] = sgb * detJ * Ji[b][a] + lj[(a * 3 + b) * g.N + p.n];
  // F = J^{-1} Fc: Jib[i][a] = Fb[i] Fc[a]; Jb -= J^{-T} Jib J^{-T}
  const double Fc[3] = {F0, F1, F2};
  double Fb[3];
  for (int i = 0; i < 3; ++i) Fb[i] = lgv[(G_F + i) * g.N + p.n];
  for (int pp = 0; pp < 3; ++pp)
    for (int q = 0; q < 3; ++q) {
      double s = 0;
      for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) s += Ji[i][pp] * Fb[i] * Fc[a] * Ji[q][a];
      Jb[pp][q] -= s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) lJe[(a * 3 + b) * NE + e] = Jb[a][b];
}

// lwe(y) on layers [0, ny-1] = transposed D (the G stencil) of ldg.
__global__ __launch_bounds__(BX * BY) void k_adjg_w(Grid g, const double* __restrict__ ldg, double* __restrict__ lwe) {
  const int i = blockIdx.x * BX + threadIdx.x, je = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int j = je - 3;
  if (i >= g.nx || j < 0 || j > g.ny - 1) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 1; l < Q; ++l) {
    const int jx = j - cy(l);  // source node x = y - c_l (fluid layers 1..ny-2)
    if (jx < 1 || jx > g.ny - 2) continue;
    const long long m = nidx(g, wrapa(i - cx(l), g.nx), jx - 1, wrapa(k - cz(l), g.nz));
    const double fct = 3.0 * wgt(l);
    for (int q = 0; q < 6; ++q)
      acc[q] += fct * (cx(l) * ldg[(0 * 6 + q) * g.N + m] + cy(l) * ldg[(1 * 6 + q) * g.N + m] +
                       cz(l) * ldg[(2 * 6 + q) * g.N + m]);
  }
  const long long e = eix(g, i, j, k);
  for (int q = 0; q < 6; ++q) lwe[q * NE + e] = acc[q];
}

// Transpose of out(x) = (1 + s) in(x) - sum_l w_l in(x + c_l), out on layers
// [olo, ohi]:  inb(y) += (1 + s) outb(y) [y in range] - sum_l w_l outb(y - c_l)
// [y - c_l in range], for y on layers [olo - 1, ohi + 1].  Adds into inb.
__global__ __launch_bounds__(BX * BY) void k_adjg_smooth(Grid g, int ncomp, int olo, int ohi, const double* __restrict__ outb,
                              double* __restrict__ inb) {
  const int i = blockIdx.x * BX + threadIdx.x, je = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int j = je - 3;
  if (i >= g.nx || j < olo - 1 || j > ohi + 1) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const long long e = eix(g, i, j, k);
  double s_all = 0;
  for (int l = 1; l < Q; ++l) s_all += wgt(l);
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0;
    if (j >= olo && j <= ohi) acc += (1.0 + s_all) * outb[c * NE + e];
    for (int l = 1; l < Q; ++l) {
      const int jx = j - cy(l);
      if (jx < olo || jx > ohi) continue;
      acc -= wgt(l) * outb[c * NE + eix(g, wrapa(i - cx(l), g.nx), jx, wrapa(k - cz(l), g.nz))];
    }
    inb[c * NE + e] += acc;
  }
}

// g = J^T J on layers [-1, ny]: lJe += from lge (J recomputed from v).
__global__ __launch_bounds__(BX * BY) void k_adjg_J(Grid g, const double* __restrict__ v, const double* __restrict__ lge,
                         double* __restrict__ lJe) {
  const int i = blockIdx.x * BX + threadIdx.x, je = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int j = je - 3;
  if (i >= g.nx || j < -1 || j > g.ny) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const long long e = eix(g, i, j, k);
  double J[3][3];
  for (int a = 0; a < 3; ++a) {
    double s[3] = {0, 0, 0};
    for (int l = 1; l < Q; ++l) {
      const double fv = v[a * NE + eix(g, wrapa(i + cx(l), g.nx), j + cy(l), wrapa(k + cz(l), g.nz))];
      s[0] += wgt(l) * cx(l) * fv;
      s[1] += wgt(l) * cy(l) * fv;
      s[2] += wgt(l) * cz(l) * fv;
    }
    for (int b = 0; b < 3; ++b) J[a][b] = (a == b ? 1.0 : 0.0) + 3.0 * s[b];
  }
  const bool fluid = j >= 1 && j <= g.ny - 2;
  double Jb[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Jb[a][b] = fluid ? lJe[(a * 3 + b) * NE + e] : 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const double lb = lge[sym(a, b) * NE + e];
      for (int c = 0; c < 3; ++c) {
        Jb[c][a] += lb * J[c][b];
        Jb[c][b] += lb * J[c][a];
      }
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) lJe[(a * 3 + b) * NE + e] = Jb[a][b];
}

// J = I + G v on layers [-1, ny]: lve(y) for y on [-2, ny+1].
__global__ __launch_bounds__(BX * BY) void k_adjg_v(Grid g, const double* __restrict__ lJe, double* __restrict__ lve) {
  const int i = blockIdx.x * BX + threadIdx.x, je = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int j = je - 3;
  if (i >= g.nx || j < -2 || j > g.ny + 1) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  double acc[3] = {0, 0, 0};
  for (int l = 1; l < Q; ++l) {
    const int jx = j - cy(l);
    if (jx < -1 || jx > g.ny) continue;
    const long long m = eix(g, wrapa(i - cx(l), g.nx), jx, wrapa(k - cz(l), g.nz));
    const double fct = 3.0 * wgt(l);
    for (int a = 0; a < 3; ++a)
      acc[a] += fct * (cx(l) * lJe[(a * 3 + 0) * NE + m] + cy(l) * lJe[(a * 3 + 1) * NE + m] +
                       cz(l) * lJe[(a * 3 + 2) * NE + m]);
  }
  const long long e = eix(g, i, j, k);
  for (int a = 0; a < 3; ++a) lve[a * NE + e] = acc[a];
}

// Chart adjoint from the displacement adjoint on the extended grid: layers
// 0..ny-1 directly, plus the transposed cubic continuation.
__global__ __launch_bounds__(BX * BY) void k_adjg_chart(Grid g, const double* __restrict__ lue, double* __restrict__ gc) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx, NC = (long long)g.nz * g.ny * g.nx;
  // u(-d) = sum_m C[d][m] u(m); u(ny-1+d) = sum_m C[d][m] u(ny-1-m)
  const double C[3][4] = {{4, -6, 4, -1}, {10, -20, 15, -4}, {20, -45, 36, -10}};
  for (int a = 0; a < 3; ++a) {
    double acc = lue[a * NE + eix(g, i, j, k)];
    if (j <= 3)
      for (int d = 0; d < 3; ++d) acc += C[d][j] * lue[a * NE + eix(g, i, -1 - d, k)];
    if (j >= g.ny - 4)
      for (int d = 0; d < 3; ++d) acc += C[d][g.ny - 1 - j] * lue[a * NE + eix(g, i, g.ny + d, k)];
    gc[a * NC + ((long long)k * g.ny + j) * g.nx + i] = acc;
  }
}

// Top-wall displacement adjoint: chart_y = xi_y + (eta/H) d_top + ...
__global__ __launch_bounds__(BX * BY) void k_adjg_disp(Grid g, const double* __restrict__ gc, double* __restrict__ gd) {
  const int i = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  const long long NC = (long long)g.nz * g.ny * g.nx;
  double acc = 0;
  for (int j = 0; j < g.ny; ++j) acc += ((j - 0.5) / g.H) * gc[NC + ((long long)k * g.ny + j) * g.nx + i];
  gd[(long long)k * g.nx + i] = acc;
}

// Save the context's current state (populations, then history) to dst.
hipError_t save_state(const Fields& F, double* dst, hipStream_t s) {
  const size_t np = sizeof(double) * 19 * (size_t)F.g.N, nh = sizeof(double) * H_N * (size_t)F.g.N;
  hipError_t e = hipMemcpyAsync(dst, F.pop[F.cur], np, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dst + 19 * F.g.N, F.hist[F.cur], nh, hipMemcpyDeviceToDevice, s);
  return e;
}

// One FP64 step from the stored state `in` (populations 19N, then history
// 10N) into `out`, leaving the context's own state buffers untouched.  With
// mom != nullptr the step also writes rho, rho u of `in` there when the
// fused step runs (*wrote says whether it did).
hipError_t step_into(Fields& F, const double* in, double* out, hipStream_t s, double tau, double* mom = nullptr,
                     bool* wrote = nullptr) {
  const size_t Nn = (size_t)F.g.N;
  void* const pop[2] = {F.pop[0], F.pop[1]};
  void* const hist[2] = {F.hist[0], F.hist[1]};
  const int cur = F.cur;
  F.pop[cur] = (void*)in;
  F.hist[cur] = (void*)(in + 19 * Nn);
  F.pop[cur ^ 1] = out;
  F.hist[cur ^ 1] = out + 19 * Nn;
  const bool with_mom = mom && step_is_fused(F) && !F.g.pj && !F.g.open;
  const hipError_t e = with_mom ? launch_step_fused_moments<double>(F, s, tau, mom) : launch_step<double>(F, s, tau);
  if (wrote) *wrote = with_mom && e == hipSuccess;
  for (int b = 0; b < 2; ++b) {
    F.pop[b] = pop[b];
    F.hist[b] = hist[b];
  }
  F.cur = cur;
  return e;
}

}  // namespace

#define HCHK(x)                        \
  do {                                 \
    hipError_t _e = (x);               \
    if (_e != hipSuccess) return _e;   \
  } while (0)

hipError_t adjoint_forward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                           double* forces) {
  const size_t state = (size_t)(19 + H_N) * F.g.N;
  HCHK(save_state(F, A.ckpt, s));
  for (int t = 0; t < K; ++t) {
    HCHK(launch_step<double>(F, s, tau));
    HCHK(launch_wall_force<double>(F, s, wall, tau, forces + 3 * t, nullptr));
    if ((t + 1) % N == 0 && t + 1 < K) HCHK(save_state(F, A.ckpt + state * ((t + 1) / N), s));
  }
  HCHK(save_state(F, A.ckpt + state * (A.nckpt - 1), s));
  return hipGetLastError();
}

hipError_t adjoint_backward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                            const double Fc[3], const double* dLdF, double* grad_disp, double* grad_chart,
                            double* grad_f0) {
  const Grid g = F.g;
  const size_t Nn = (size_t)g.N;
  const size_t state = (size_t)(19 + H_N) * Nn;
  const size_t NE = (size_t)g.nz * (g.ny + 6) * g.nx, NC = (size_t)g.nz * g.ny * g.nx;
  const dim3 b(BX, BY), fg = fluid_grid(g), cg = col_grid(g), eg = ext_grid(g);
  // the node kernel runs one wave per SIMD: one-wave workgroups let each
  // SIMD take the next one as soon as its own wave ends
  const dim3 nb(BX, 1), ng(row_group_blocks(g));
  double* mom = (double*)F.mom;
  const double* geo = (const double*)F.geo;
  int cur = 0;
  HCHK(hipMemsetAsync(A.lf[cur], 0, sizeof(double) * 19 * Nn, s));
  HCHK(hipMemsetAsync(A.lp[cur], 0, sizeof(double) * H_N * Nn, s));
  HCHK(hipMemsetAsync(A.lg, 0, sizeof(double) * G_N * Nn, s));
  HCHK(hipMemsetAsync(A.lj, 0, sizeof(double) * 9 * Nn, s));
  HCHK(hipMemsetAsync(A.ub, 0, sizeof(double) * 6 * (size_t)g.nz * g.nx, s));
  const double* uwd = (const double*)F.uw;
  const int mv0 = F.moving[0], mv1 = F.moving[1];
  const bool mw = mv0 || mv1;
  // force at the final state K
  {
    const double* fin = A.ckpt + state * (A.nckpt - 1);
    hipLaunchKernelGGL(k_adj_force, cg, b, 0, s, g, wall, fin, fin + 19 * Nn, geo, (const double*)F.jac, tau,
                       dLdF + 3 * (K - 1), A.lf[cur], A.lg, A.lj);
  }
  const int nseg = (K + N - 1) / N;
  std::vector<char> have_mom((size_t)N, 0);  // moments of the segment's state t0 + i kept in A.tmom slot i
  for (int sgm = nseg - 1; sgm >= 0; --sgm) {
    const int t0 = sgm * N, t1 = (t0 + N < K) ? t0 + N : K;
    // states t0..t1-1 of the segment: its checkpoint, then traj slots 1..
    auto at = [&](int t) { return t == t0 ? A.ckpt + state * sgm : A.traj + state * (t - t0); };
    // the recompute steps also leave the moments of the states they step from
    for (int t = t0; t + 1 < t1; ++t) {
      bool wrote = false;
      HCHK(step_into(F, at(t), at(t + 1), s, tau, A.tmom + 4 * Nn * (t - t0), &wrote));
      have_mom[t - t0] = wrote;
    }
    have_mom[t1 - 1 - t0] = false;  // the segment's last state is no step's input
    for (int t = t1 - 1; t >= t0; --t) {
      const double* st = at(t);
      const double* pop = st;
      const double* hist = st + 19 * Nn;
      const double* mt = mom;
      if (have_mom[t - t0])
        mt = A.tmom + 4 * Nn * (t - t0);
      else
        hipLaunchKernelGGL(k_adj_moments, fg, b, 0, s, g, pop, hist, geo, mom);
      // the force of state t (t >= 1, in the loss) is reversed inside its node kernel
      const double* W = t >= 1 ? dLdF + 3 * (t - 1) : nullptr;
      hipLaunchKernelGGL(mw ? k_adj_node<true> : k_adj_node<false>, ng, nb, 0, s, g, 0, pop, hist, geo, mt, tau,
                         (const double*)A.lf[cur], (const double*)A.lp[cur], A.lpb, A.lml, A.ldj, A.lp[cur ^ 1],
                         A.lg, uwd, mv0, mv1, A.ub, wall, W, (const double*)F.jac, A.lj);
      hipLaunchKernelGGL(mw ? k_adj_gather<true> : k_adj_gather<false>, fg, b, 0, s, g, geo, mt,
                         (const double*)A.lf[cur], tau, (const double*)A.lpb, (const double*)A.lml,
                         (const double*)A.ldj, (const double*)nullptr, A.lf[cur ^ 1], A.lg, uwd, mv0, mv1, A.ub);
      cur ^= 1;
    }
  }
  // history of the initial state: F(x,-1) := F(state 0)
  {
    const double* pop = A.ckpt;
    const double* hist = A.ckpt + 19 * Nn;
    // state 0 starts segment 0, the last one swept: its moments are in slot 0 if kept
    const double* mt = mom;
    if (have_mom[0])
      mt = A.tmom;
    else
      hipLaunchKernelGGL(k_adj_moments, fg, b, 0, s, g, pop, hist, geo, mom);
    hipLaunchKernelGGL(mw ? k_adj_node<true> : k_adj_node<false>, ng, nb, 0, s, g, 1, pop, hist, geo, mt, tau,
                       (const double*)A.lf[cur], (const double*)A.lp[cur], A.lpb, A.lml, A.ldj, (double*)nullptr,
                       A.lg, uwd, mv0, mv1, A.ub, wall, (const double*)nullptr, (const double*)F.jac, A.lj);
    hipLaunchKernelGGL(mw ? k_adj_gather<true> : k_adj_gather<false>, fg, b, 0, s, g, geo, mt,
                       (const double*)nullptr, tau, (const double*)A.lpb, (const double*)A.lml,
                       (const double*)A.ldj, (const double*)A.lf[cur], A.lf[cur ^ 1], A.lg, uwd, mv0, mv1, A.ub);
    cur ^= 1;
  }
  if (grad_f0) HCHK(hipMemcpyAsync(grad_f0, A.lf[cur], sizeof(double) * 19 * Nn, hipMemcpyDeviceToDevice, s));
  // moving walls: their chart-component velocity depends on J at the wall nodes
  if (mv0 || mv1)
    hipLaunchKernelGGL(k_adj_wall_velocity, cg, b, 0, s, g, (const double*)F.jac, uwd, mv0, mv1,
                       (const double*)A.ub, A.lj);
  // geometry
  if (grad_disp || grad_chart) {
    HCHK(hipMemsetAsync(A.lge, 0, sizeof(double) * 6 * NE, s));
    HCHK(hipMemsetAsync(A.lJe, 0, sizeof(double) * 9 * NE, s));
    HCHK(hipMemsetAsync(A.lve, 0, sizeof(double) * 3 * NE, s));
    HCHK(hipMemsetAsync(A.lue, 0, sizeof(double) * 3 * NE, s));
    hipLaunchKernelGGL(k_adjg_fluid, fg, b, 0, s, g, (const double*)F.wext,
                       (const double*)F.jac, Fc[0], Fc[1], Fc[2], (const double*)A.lg, (const double*)A.lj, A.ldg,
                       A.lge, A.lJe);
    hipLaunchKernelGGL(k_adjg_w, eg, b, 0, s, g, (const double*)A.ldg, A.lwe);
    hipLaunchKernelGGL(k_adjg_smooth, eg, b, 0, s, g, 6, 0, g.ny - 1, (const double*)A.lwe, A.lge);
    hipLaunchKernelGGL(k_adjg_J, eg, b, 0, s, g, (const double*)F.vtmp, (const double*)A.lge, A.lJe);
    hipLaunchKernelGGL(k_adjg_v, eg, b, 0, s, g, (const double*)A.lJe, A.lve);
    hipLaunchKernelGGL(k_adjg_smooth, eg, b, 0, s, g, 3, -2, g.ny + 1, (const double*)A.lve, A.lue);
    hipLaunchKernelGGL(k_adjg_chart, dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz), b, 0, s, g,
                       (const double*)A.lue, A.gc);
    if (grad_chart) HCHK(hipMemcpyAsync(grad_chart, A.gc, sizeof(double) * 3 * NC, hipMemcpyDeviceToDevice, s));
    if (grad_disp) hipLaunchKernelGGL(k_adjg_disp, cg, b, 0, s, g, (const double*)A.gc, grad_disp);
  }
  // The segments were rebuilt in the trajectory slots: the context's state
  // is still the one lbm_forward_record ended with.
  return hipGetLastError();
}

}  // namespace lbm
