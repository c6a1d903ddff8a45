// One time step of the curved-space D3Q19 scheme, and the kernels that move
// state in and out.
//
// Storage ("pull" layout): pop[l][x] holds the post-collision deviation
// f*_l(x) - w_l of node x, except on links that leave the fluid through a
// wall, where it holds the bounced value f*_l - 2 (w_l/sqrt g) rho (c_l.u_w)/c_s^2
// destined to come back to x as direction opp(l).  The streamed value of
// Eq. (streaming) at node x is therefore
//   g_l(x) = pop[l][x - c_l]   if x - c_l is a fluid node,
//          = pop[opp(l)][x]    otherwise (halfway bounce-back),
// and f_l(x, t) = g_l(x) + F_l(x, t-1)/2, with F(x, t-1) rebuilt from the ten
// history coefficients of x.  Reads are shifted by at most one node in each
// direction; all writes are aligned and coalesced.
//
// A step is two passes.  The lattice gradient d_k(rho u^i) (App. D, radius 1)
// needs the momentum of all 18 neighbours before any collision, so pass 1
// forms rho and rho u at every node, and pass 2 does the rest of the step
// node-locally: equilibrium, stress, forcing A/B/C, collision, bounce-back
// term, history update.
#include <mutex>

#include "lbm_internal.h"
#include "lbm_pull.h"

namespace lbm {

namespace {

__device__ __forceinline__ bool node_pos(const Grid& g, Pos& p) {
  p.i = blockIdx.x * BX + threadIdx.x;
  p.jf = blockIdx.y * BY + threadIdx.y;
  p.k = blockIdx.z;
  if (p.i >= g.nx || p.jf >= g.H) return false;
  p.n = ((long long)p.k * g.H + p.jf) * g.nx + p.i;
  return true;
}

// Columns of a launch over the m columns at each end in x: 0..m-1 and
// nx-m..nx-1, or all nx columns when those overlap.
inline __host__ __device__ int end_columns(const Grid& g, int m) { return 2 * m < g.nx ? 2 * m : g.nx; }

// Node of a launch over the grid (ends = 0: 2D tiles of the fluid grid) or
// over the m = ends columns at each end in x (a 1D launch, one thread per
// (column, row, plane), columns fastest).
__device__ __forceinline__ bool node_pos_ends(const Grid& g, int ends, Pos& p) {
  if (!ends) return node_pos(g, p);
  const int nc = end_columns(g, ends);
  const long long t = ((long long)blockIdx.x * BY + threadIdx.y) * BX + threadIdx.x;
  if (t >= (long long)nc * g.H * g.nz) return false;
  const int c = (int)(t % nc);
  const long long r = t / nc;
  p.jf = (int)(r % g.H);
  p.k = (int)(r / g.H);
  p.i = (nc < 2 * ends || c < ends) ? c : g.nx - 2 * ends + c;
  p.n = ((long long)p.k * g.H + p.jf) * g.nx + p.i;
  return true;
}

// 1D grid of BX x BY blocks covering the end-column launch of node_pos_ends.
inline dim3 ends_grid(const Grid& g, int ends) {
  const long long n = (long long)end_columns(g, ends) * g.H * g.nz;
  return dim3((unsigned)((n + BX * BY - 1) / (BX * BY)));
}

template <class T>
__device__ __forceinline__ void load_coef(const T* __restrict__ hist, long long N, long long n, Coef<T>& c) {
  c.A = hist[H_A * N + n];
#pragma unroll
  for (int a = 0; a < 3; ++a) c.B[a] = hist[(H_B + a) * N + n];
#pragma unroll
  for (int q = 0; q < 6; ++q) c.C[q] = hist[(H_C + q) * N + n];
}

template <class T>
__device__ __forceinline__ void store_coef(T* __restrict__ hist, long long N, long long n, const Coef<T>& c) {
  hist[H_A * N + n] = c.A;
#pragma unroll
  for (int a = 0; a < 3; ++a) hist[(H_B + a) * N + n] = c.B[a];
#pragma unroll
  for (int q = 0; q < 6; ++q) hist[(H_C + q) * N + n] = c.C[q];
}

// rho - 1 and rho u of the streamed state at p: rho = sqrt g sum_l g_l + A/2,
// rho u = sqrt g sum_l g_l c_l + B/2 (the half history term summed in closed
// form: sum_l F_l sqrt g = A, sum_l F_l c_l sqrt g = B).  The pulled
// deviations are left in gv.
template <class T>
__device__ __forceinline__ void streamed_moments(const T* __restrict__ pop, const T* __restrict__ hist,
                                                 const T* __restrict__ geo, const T* __restrict__ vin,
                                                 const Grid& g, const Pos& p, T& dr, T j[3], T gv[Q]) {
  pull_all(pop, hist, geo, vin, g, p, gv);
  T s = 0, j0 = 0, j1 = 0, j2 = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const T v = gv[l];
    s += v;
    if (cx(l)) j0 += T(cx(l)) * v;
    if (cy(l)) j1 += T(cy(l)) * v;
    if (cz(l)) j2 += T(cz(l)) * v;
  });
  const T sgd = geo[G_SG * g.N + p.n];
  const T sg = T(1) + sgd;
  dr = sgd + sg * s + T(0.5) * hist[H_A * g.N + p.n];
  j[0] = sg * j0 + T(0.5) * hist[(H_B + 0) * g.N + p.n];
  j[1] = sg * j1 + T(0.5) * hist[(H_B + 1) * g.N + p.n];
  j[2] = sg * j2 + T(0.5) * hist[(H_B + 2) * g.N + p.n];
}

// Second-order isotropic lattice gradient dj[k][i] = (1/c_s^2) sum_l w_l c_l^k
// j^i(x + c_l) (App. D).  Neighbours in a wall layer carry the mirror ghost
// j = 2 rho_m u_w - j_m of the fluid node m in the same column next to the wall;
// a neighbour across the plate is replaced in the same way by the ghost of the
// node m on this side in the neighbour's column, with the plate velocity.
// PL: the grid has a plate; MV: a wall moves.  Each combination has its own
// unrolled loop, so the common one (neither) has no branch between the
// neighbours' loads.
template <class T, bool PL, bool MV>
__device__ __forceinline__ void lattice_gradient_t(const T* __restrict__ mom, const T* __restrict__ uw, const int mv0,
                                                   const int mv1, const T* __restrict__ up, const Grid& g,
                                                   const Pos& p, T dj[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dj[a][b] = T(0);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    if (l == 0) return;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    // beyond an open end: the end column itself (zero gradient)
    const int in = !x ? p.i : (g.open ? min(max(p.i + x, 0), g.nx - 1) : wrapd(p.i + x, g.nx));
    const int kn = z ? wrapd(p.k + z, g.nz) : p.k;
    const int jn = p.jf + y;
    // No branch around the loads: a cut link (plate) or a solid neighbour
    // (wall) reads this layer's node for its mirror ghost 2 rho u - j, a
    // fluid neighbour its own j; the choice is of address and sign.
    const bool cutp = PL && plate_cut(g, p.i, p.jf, x, y);
    const bool fluid = y == 0 || (jn >= 0 && jn < g.H);
    const bool ghost = cutp || !fluid;
    const long long m = ((long long)kn * g.H + (ghost ? p.jf : jn)) * g.nx + in;
    const T sgn = ghost ? T(-1) : T(1);
    T jb[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) jb[b] = sgn * mom[(1 + b) * g.N + m];
    if constexpr (y != 0 && (PL || MV)) {
      const T r2 = T(2) * (T(1) + mom[m]);
      if constexpr (PL) {
        const long long c = (((long long)(p.jf == g.pj ? 1 : 0) * g.nz + kn) * g.nx + in) * 3;
        const T rc = cutp ? r2 : T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) jb[b] += rc * up[c + b];
      }
      if constexpr (MV) {
        const int w = jn < 0 ? 0 : 1;
        const bool mvw = !fluid && (w == 0 ? mv0 : mv1);
        const long long c = (((long long)w * g.nz + kn) * g.nx + in) * 3;
        const T rw = mvw ? r2 : T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) jb[b] += rw * uw[c + b];
      }
    }
    constexpr T f = T(3.0 * wgt(l));
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (x) dj[0][b] += T(x) * f * jb[b];
      if (y) dj[1][b] += T(y) * f * jb[b];
      if (z) dj[2][b] += T(z) * f * jb[b];
    }
  });
}

template <class T>
__device__ __forceinline__ void lattice_gradient(const T* __restrict__ mom, const T* __restrict__ uw, const int mv0,
                                                 const int mv1, const T* __restrict__ up, const Grid& g,
                                                 const Pos& p, T dj[3][3]) {
  const bool mv = mv0 || mv1;
  if (g.pj) {
    if (mv)
      lattice_gradient_t<T, true, true>(mom, uw, mv0, mv1, up, g, p, dj);
    else
      lattice_gradient_t<T, true, false>(mom, uw, mv0, mv1, up, g, p, dj);
  } else {
    if (mv)
      lattice_gradient_t<T, false, true>(mom, uw, mv0, mv1, up, g, p, dj);
    else
      lattice_gradient_t<T, false, false>(mom, uw, mv0, mv1, up, g, p, dj);
  }
}

// ---------------------------------------------------------------- pass 1
template <class T>
__global__ __launch_bounds__(BX* BY) void k_moments(Grid g, int ends, const T* __restrict__ pop,
                                                   const T* __restrict__ hist, const T* __restrict__ geo,
                                                   const T* __restrict__ vin, T* __restrict__ mom) {
  Pos p;
  if (!node_pos_ends(g, ends, p)) return;
  T dr, j[3], gv[Q];
  streamed_moments(pop, hist, geo, vin, g, p, dr, j, gv);
  mom[p.n] = dr;
  mom[g.N + p.n] = j[0];
  mom[2 * g.N + p.n] = j[1];
  mom[3 * g.N + p.n] = j[2];
}

// ---------------------------------------------------------------- pass 2
// Collision f* = f - (f - feq)/tau + F(t) - F(t-1)/2 (Eq. collision with the
// leading f restored) and the bounce-back term of Eq. (streaming) at walls.
template <class T>
__global__ __launch_bounds__(BX* BY) void k_collide(Grid g, int ends, const T* __restrict__ pin, T* __restrict__ pout,
                                                   const T* __restrict__ hist, T* __restrict__ hout,
                                                   const T* __restrict__ geo,
                                                   const T* __restrict__ mom, const T* __restrict__ uw, int mv0,
                                                   int mv1, const T* __restrict__ up, const T* __restrict__ vin,
                                                   T tau, int* __restrict__ flag) {
  Pos p;
  if (!node_pos_ends(g, ends, p)) return;
  NodeGeo<T> G;
  load_geo(geo, g.N, p.n, G);
  Coef<T> cp;
  load_coef(hist, g.N, p.n, cp);
  const T sg = T(1) + G.sgd, isg = T(1) / sg;
  T Fp[Q], ft[Q];
  forcing_pops(cp, isg, Fp);
  pull_all(pin, hist, geo, vin, g, p, ft);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    ft[l] += T(0.5) * Fp[l];
  });
  const T dr = mom[p.n];
  const T j[3] = {mom[g.N + p.n], mom[2 * g.N + p.n], mom[3 * g.N + p.n]};
  T dj[3][3];
  lattice_gradient(mom, uw, mv0, mv1, up, g, p, dj);
  T ne[Q], Tm[6];
  node_stress(G, ft, dr, j, tau, ne, Tm);
  Coef<T> c;
  forcing_coef(G, j, Tm, dj, c);
  T F[Q];
  forcing_pops(c, isg, F);
  const T rho = T(1) + dr;
  const T itau = T(1) / tau;
  const long long col0 = ((long long)p.k * g.nx + p.i) * 3;
  T chk = T(0);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    T v = ft[l] - ne[l] * itau + F[l] - T(0.5) * Fp[l];
    constexpr int y = cy(l);
    if ((y > 0 && p.jf == g.H - 1) || (y < 0 && p.jf == 0)) {
      const int w = y > 0 ? 1 : 0;
      if (w == 0 ? mv0 : mv1) {
        const T* u = uw + (long long)w * g.nz * g.nx * 3 + col0;
        T cu = T(0);
        if (cx(l)) cu += T(cx(l)) * u[0];
        cu += T(y) * u[1];
        if (cz(l)) cu += T(cz(l)) * u[2];
        v -= T(6.0 * wgt(l)) * isg * rho * cu;
      }
    }
    if (plate_cut(g, p.i, p.jf, cx(l), y)) {
      const T* u = up + (((long long)(p.jf == g.pj ? 1 : 0) * g.nz + p.k) * g.nx + p.i) * 3;
      T cu = T(y) * u[1];
      if (cx(l)) cu += T(cx(l)) * u[0];
      if (cz(l)) cu += T(cz(l)) * u[2];
      v -= T(6.0 * wgt(l)) * isg * rho * cu;
    }
    chk += v;
    pout[(long long)l * g.N + p.n] = v;
  });
  store_coef(hout, g.N, p.n, c);
  const T uu = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
  if (!(rho > T(0)) || !(uu < T(0.1) * rho * rho) || !isfinite(chk)) atomicOr(flag, 1);
}

// ------------------------------------------------------- state in / out
// Equilibrium state in FP64: f = w + feq deviations of (rho, J^{-1} u_cart).
template <class T>
__global__ __launch_bounds__(BX * BY) void k_feq_full(Grid g, const double* __restrict__ rho_in, const double* __restrict__ uc,
                           const double* __restrict__ jac, const T* __restrict__ geo, double* __restrict__ full) {
  Pos p;
  if (!node_pos(g, p)) return;
  NodeGeo<double> G;
  G.sgd = (double)geo[G_SG * g.N + p.n];
#pragma unroll
  for (int q = 0; q < 6; ++q) G.gid[q] = (double)geo[(G_GI + q) * g.N + p.n];
  double J[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + p.n];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double Ji[3][3] = {
      {(J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det,
       (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det},
      {(J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det,
       (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det},
      {(J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det,
       (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det}};
  const double r = rho_in ? rho_in[p.n] : 1.0;
  double u[3] = {0, 0, 0};
  if (uc) {
    const double v[3] = {uc[p.n], uc[g.N + p.n], uc[2 * g.N + p.n]};
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = Ji[a][0] * v[0] + Ji[a][1] * v[1] + Ji[a][2] * v[2];
  }
  const double j[3] = {r * u[0], r * u[1], r * u[2]};
  double fe[Q];
  equilibrium_dev(G, r - 1.0, j, fe);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    full[(long long)l * g.N + p.n] = wgt(l) + fe[l];
  });
}

// Moments of a full FP64 state f (rho = sqrt g sum f, j = sqrt g sum f c).
template <class T>
__global__ __launch_bounds__(BX * BY) void k_moments_full(Grid g, const double* __restrict__ f, const T* __restrict__ geo, T* __restrict__ mom) {
  Pos p;
  if (!node_pos(g, p)) return;
  double s = 0, j0 = 0, j1 = 0, j2 = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const double v = f[(long long)l * g.N + p.n] - wgt(l);
    s += v;
    if (cx(l)) j0 += cx(l) * v;
    if (cy(l)) j1 += cy(l) * v;
    if (cz(l)) j2 += cz(l) * v;
  });
  const double sgd = (double)geo[G_SG * g.N + p.n], sg = 1.0 + sgd;
  mom[p.n] = (T)(sgd + sg * s);
  mom[g.N + p.n] = (T)(sg * j0);
  mom[2 * g.N + p.n] = (T)(sg * j1);
  mom[3 * g.N + p.n] = (T)(sg * j2);
}

// Forcing history of a full state (the forcing F(x, 0) that stands in for
// F(x, -1) at the first step).
template <class T>
__global__ __launch_bounds__(BX * BY) void k_hist_full(Grid g, const double* __restrict__ f, const T* __restrict__ geo, const T* __restrict__ mom,
                            const T* __restrict__ uw, int mv0, int mv1, const T* __restrict__ up, T tau,
                            T* __restrict__ hist) {
  Pos p;
  if (!node_pos(g, p)) return;
  NodeGeo<T> G;
  load_geo(geo, g.N, p.n, G);
  T ft[Q];
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    ft[l] = (T)(f[(long long)l * g.N + p.n] - wgt(l));
  });
  const T dr = mom[p.n];
  const T j[3] = {mom[g.N + p.n], mom[2 * g.N + p.n], mom[3 * g.N + p.n]};
  T dj[3][3];
  lattice_gradient(mom, uw, mv0, mv1, up, g, p, dj);
  T ne[Q], Tm[6];
  node_stress(G, ft, dr, j, tau, ne, Tm);
  Coef<T> c;
  forcing_coef(G, j, Tm, dj, c);
  store_coef(hist, g.N, p.n, c);
}

// In place: full[l] = f_l - w_l - F_l(history)/2, the streamed deviation g~.
template <class T>
__global__ __launch_bounds__(BX * BY) void k_full_to_streamed(Grid g, double* __restrict__ full, const T* __restrict__ hist,
                                   const T* __restrict__ geo) {
  Pos p;
  if (!node_pos(g, p)) return;
  Coef<T> c;
  load_coef(hist, g.N, p.n, c);
  const T isg = T(1) / (T(1) + geo[G_SG * g.N + p.n]);
  T Fp[Q];
  forcing_pops(c, isg, Fp);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const long long q = (long long)l * g.N + p.n;
    full[q] = full[q] - wgt(l) - 0.5 * (double)Fp[l];
  });
}

// Inverse of the pull: pop[l][y] = g~_l(y + c_l) if the link from y to
// y + c_l is open, else (through a wall or the plate) g~_opp(l)(y).  With
// open ends in x the slots of links leaving through an end are never read
// (the values arriving there are extrapolated), so their periodic image
// does no harm.
template <class T>
__global__ __launch_bounds__(BX * BY) void k_unpull(Grid g, const double* __restrict__ gs, T* __restrict__ pop) {
  Pos p;
  if (!node_pos(g, p)) return;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    const int jd = p.jf + y;
    double v;
    if (jd < 0 || jd >= g.H || plate_cut(g, p.i, p.jf, x, y)) {
      v = gs[(long long)opp(l) * g.N + p.n];
    } else {
      const int id = x ? wrapd(p.i + x, g.nx) : p.i;
      const int kd = z ? wrapd(p.k + z, g.nz) : p.k;
      v = gs[(long long)l * g.N + ((long long)kd * g.H + jd) * g.nx + id];
    }
    pop[(long long)l * g.N + p.n] = (T)v;
  });
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_get_pops(Grid g, const T* __restrict__ pop, const T* __restrict__ hist, const T* __restrict__ geo,
                           const T* __restrict__ vin, double* __restrict__ out) {
  Pos p;
  if (!node_pos(g, p)) return;
  Coef<T> c;
  load_coef(hist, g.N, p.n, c);
  const T isg = T(1) / (T(1) + geo[G_SG * g.N + p.n]);
  T Fp[Q], gv[Q];
  forcing_pops(c, isg, Fp);
  pull_all(pop, hist, geo, vin, g, p, gv);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    out[(long long)l * g.N + p.n] = wgt(l) + ((double)gv[l] + 0.5 * (double)Fp[l]);
  });
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_get_hist(Grid g, const T* __restrict__ hist, double* __restrict__ out) {
  Pos p;
  if (!node_pos(g, p)) return;
  for (int q = 0; q < H_N; ++q) out[q * g.N + p.n] = (double)hist[q * g.N + p.n];
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_get_geo(Grid g, const T* __restrict__ geo, double* __restrict__ out) {
  Pos p;
  if (!node_pos(g, p)) return;
  for (int q = 0; q < G_N; ++q) {
    double v = (double)geo[q * g.N + p.n];
    if (q == G_SG || q == G_GI + 0 || q == G_GI + 3 || q == G_GI + 5) v += 1.0;
    out[q * g.N + p.n] = v;
  }
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_moments_out(Grid g, const T* __restrict__ pop, const T* __restrict__ hist, const T* __restrict__ geo,
                              const T* __restrict__ vin, const double* __restrict__ jac, double* __restrict__ rho,
                              double* __restrict__ u, int cart) {
  Pos p;
  if (!node_pos(g, p)) return;
  T dr, j[3], gv[Q];
  streamed_moments(pop, hist, geo, vin, g, p, dr, j, gv);
  const double r = 1.0 + (double)dr;
  if (rho) rho[p.n] = r;
  if (u) {
    const double v[3] = {(double)j[0] / r, (double)j[1] / r, (double)j[2] / r};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double s = v[a];
      if (cart)
        s = jac[(a * 3 + 0) * g.N + p.n] * v[0] + jac[(a * 3 + 1) * g.N + p.n] * v[1] +
            jac[(a * 3 + 2) * g.N + p.n] * v[2];
      u[a * g.N + p.n] = s;
    }
  }
}

// Node-exact traction sqrt g T^{i y} e_i (Cartesian) at fluid node p, times
// sgn, added to t.
template <class T>
__device__ __forceinline__ void node_traction(const Grid& g, const T* __restrict__ pop, const T* __restrict__ hist,
                                              const T* __restrict__ geo, const T* __restrict__ vin,
                                              const double* __restrict__ jac, T tau, const Pos& p, double sgn,
                                              double t[3]) {
  NodeGeo<T> G;
  load_geo(geo, g.N, p.n, G);
  Coef<T> cp;
  load_coef(hist, g.N, p.n, cp);
  const T isg = T(1) / (T(1) + G.sgd);
  T Fp[Q], ft[Q];
  forcing_pops(cp, isg, Fp);
  T dr, j[3];
  streamed_moments(pop, hist, geo, vin, g, p, dr, j, ft);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    ft[l] += T(0.5) * Fp[l];
  });
  T ne[Q], Tm[6];
  node_stress(G, ft, dr, j, tau, ne, Tm);
  const double sg = 1.0 + (double)G.sgd;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
#pragma unroll
    for (int i2 = 0; i2 < 3; ++i2) s += (double)Tm[sym(i2, 1)] * jac[(a * 3 + i2) * g.N + p.n];
    t[a] += sgn * sg * s;
  }
}

// Momentum exchange at a wall at rest, per column: the populations that
// streamed into the wall in the last step came back reversed, each handing
// the wall 2 f*_l c_l; their post-collision values sit in the bounce-back
// slots (f*_l = w_l + pop[l] at the fluid node next to the wall).  Cartesian
// 2 sqrt g J c_l f*_l, added to t.
template <class T>
__device__ __forceinline__ void node_exchange(const Grid& g, int wall, const T* __restrict__ pop,
                                              const T* __restrict__ geo, const double* __restrict__ jac,
                                              const Pos& p, double t[3]) {
  const double sg = 1.0 + (double)geo[G_SG * g.N + p.n];
  double J[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + p.n];
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int y = cy(l);
    if ((wall == 1 && y > 0) || (wall == 0 && y < 0)) {
      const double fs = wgt(l) + (double)pop[(long long)l * g.N + p.n];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double v = J[a][1] * y;
        if (cx(l)) v += J[a][0] * cx(l);
        if (cz(l)) v += J[a][2] * cz(l);
        t[a] += 2.0 * sg * fs * v;
      }
    }
  });
}

// Sum of v over the 64 lanes of a wave by a butterfly of lane exchanges.
// Floating-point addition is commutative, so every lane ends with the same,
// launch-independent value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Force per column on a wall (wall 0 / 1: the traction at the fluid layer
// next to it, outward-normal sign, or with mem != 0 the momentum exchange) or
// on the plate (wall 2: the traction of both faces in the plate columns, + at
// the node below and - at the node above; zero in the other columns), and
// its sum over the columns, in one launch (one column per thread).  Each wave
// sums its columns by lane exchanges, the block adds its waves' sums in wave
// order and stores the result in part[block]; the block that finishes last
// (counted in *count) adds the partials in block order and clears the
// counter for the next launch, so the total does not depend on the order the
// blocks ran in.  Only the partials are published (release before the count,
// acquire in the last block alone), so no other block's cached data is
// invalidated.
template <class T>
__global__ __launch_bounds__(WF_THREADS) void k_wall_force(Grid g, int wall, int mem, const T* __restrict__ pop,
                                                          const T* __restrict__ hist, const T* __restrict__ geo,
                                                          const T* __restrict__ vin, const double* __restrict__ jac,
                                                          T tau, double* __restrict__ per_node,
                                                          double* __restrict__ part, unsigned* __restrict__ count,
                                                          double* __restrict__ total) {
  constexpr int NW = WF_THREADS / 64;
  __shared__ double red[NW][3];
  __shared__ unsigned last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long col = (long long)blockIdx.x * WF_THREADS + tid;
  double t[3] = {0, 0, 0};
  if (col < (long long)g.nx * g.nz) {
    Pos p;
    p.i = (int)(col % g.nx);
    p.k = (int)(col / g.nx);
    if (wall < 2) {
      p.jf = wall == 0 ? 0 : g.H - 1;
      p.n = ((long long)p.k * g.H + p.jf) * g.nx + p.i;
      if (mem)
        node_exchange(g, wall, pop, geo, jac, p, t);
      else
        node_traction(g, pop, hist, geo, vin, jac, tau, p, wall == 0 ? -1.0 : 1.0, t);
    } else if (p.i >= g.pi0 && p.i <= g.pi1) {
      for (int side = 0; side < 2; ++side) {
        p.jf = g.pj - 1 + side;
        p.n = ((long long)p.k * g.H + p.jf) * g.nx + p.i;
        node_traction(g, pop, hist, geo, vin, jac, tau, p, side == 0 ? 1.0 : -1.0, t);
      }
    }
    if (per_node) {
#pragma unroll
      for (int a = 0; a < 3; ++a) per_node[col * 3 + a] = t[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) t[a] = wave_sum(t[a]);
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) red[wave][a] = t[a];
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double s = red[0][a];
#pragma unroll
      for (int w = 1; w < NW; ++w) s += red[w][a];
      part[(size_t)blockIdx.x * 3 + a] = s;
    }
    // publish the partial, then count this block as done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    last = atomicAdd(count, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last || wave != 0) return;
  // every other block's partial is visible past this point
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double s[3] = {0, 0, 0};
  for (unsigned b = lane; b < gridDim.x; b += 64)
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] += part[(size_t)b * 3 + a];
#pragma unroll
  for (int a = 0; a < 3; ++a) s[a] = wave_sum(s[a]);
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) total[a] = s[a];
    *count = 0u;
  }
}

}  // namespace

// Reduction scratch of the allocation-free wall force: the block partials
// (3 doubles per block) and, after them, the completion counter.
// Every context on a device shares this one array.
constexpr size_t NOALLOC_COUNT_OFF = sizeof(double) * 3 * (size_t)NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) unsigned char scratch[NOALLOC_COUNT_OFF + 256];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES];  // device address of `scratch` on each device
}  // namespace

hipError_t noalloc_scratch_init(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    // the counter must read zero before the first launch (every launch
    // leaves it at zero again)
    e = hipMemset((char*)p + NOALLOC_COUNT_OFF, 0, 256);
    if (e != hipSuccess) return e;
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

template <class T>
hipError_t launch_wall_force_noalloc(Fields& F, hipStream_t s, int wall, T tau, double* total, double* per_node,
                                     int mem, void* scr) {
  if (!scr) return hipErrorInvalidValue;
  if (wall_force_blocks(F.g) > NOALLOC_MAX_BLOCKS) return hipErrorInvalidValue;
  return launch_wall_force<T>(F, s, wall, tau, total, per_node, mem, (double*)scr,
                              (unsigned*)((char*)scr + NOALLOC_COUNT_OFF));
}

// One step; with ev != nullptr, events ev[0..2] bracket the kernels of the
// step (the fused step is one kernel: ev[1] and ev[2] then coincide).
template <class T> hipError_t launch_step(Fields& F, hipStream_t s, T tau, hipEvent_t* ev) {
  const Grid g = F.g;
  hipError_t e = hipSuccess;
  auto mark = [&](int k) {
    if (ev && e == hipSuccess) e = hipEventRecord(ev[k], s);
  };
  dim3 b(BX, BY);
  const int cur = F.cur;
  const T* pin = (const T*)F.pop[cur];
  T* pout = (T*)F.pop[cur ^ 1];
  if (step_is_fused(F)) {
    mark(0);
    if (e == hipSuccess) e = launch_step_fused<T>(F, s, tau, F.zc);
    mark(1);
    if (e == hipSuccess && g.open) {
      // The fused kernel treats x as periodic.  With open ends, the end
      // columns and their neighbours (whose gradient reads an end column's
      // momentum) are redone by the two-pass kernels over the end columns
      // only: the streamed moments of the three columns at each end with
      // the open-end rule, then the collision of the two columns at each
      // end, overwriting what the fused kernel wrote for them.
      hipLaunchKernelGGL(k_moments<T>, ends_grid(g, 3), b, 0, s, g, 3, pin, (const T*)F.hist[cur],
                         (const T*)F.geo, (const T*)F.vin, (T*)F.mom);
      hipLaunchKernelGGL(k_collide<T>, ends_grid(g, 2), b, 0, s, g, 2, pin, pout, (const T*)F.hist[cur],
                         (T*)F.hist[cur ^ 1],
                         (const T*)F.geo, (const T*)F.mom, (const T*)F.uw, F.moving[0], F.moving[1],
                         (const T*)F.up, (const T*)F.vin, tau, F.flag);
      e = hipGetLastError();
    }
    mark(2);
    return e;
  }
  mark(0);
  hipLaunchKernelGGL(k_moments<T>, fluid_grid(g), b, 0, s, g, 0, pin, (const T*)F.hist[cur], (const T*)F.geo,
                     (const T*)F.vin, (T*)F.mom);
  mark(1);
  hipLaunchKernelGGL(k_collide<T>, fluid_grid(g), b, 0, s, g, 0, pin, pout, (const T*)F.hist[cur],
                     (T*)F.hist[cur ^ 1], (const T*)F.geo,
                     (const T*)F.mom, (const T*)F.uw, F.moving[0], F.moving[1], (const T*)F.up, (const T*)F.vin, tau,
                     F.flag);
  mark(2);
  F.cur ^= 1;
  const hipError_t l = hipGetLastError();
  return e != hipSuccess ? e : l;
}

template <class T> hipError_t launch_feq_full(Fields& F, hipStream_t s, const double* rho, const double* uc) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_feq_full<T>, fluid_grid(F.g), b, 0, s, F.g, rho, uc, F.jac, (const T*)F.geo, F.full);
  return hipGetLastError();
}

// F.full holds a full FP64 state f; build history and the pull layout.
template <class T> hipError_t launch_set_state(Fields& F, hipStream_t s, const double* f, T tau) {
  const Grid g = F.g;
  dim3 b(BX, BY);
  if (f != F.full) {
    hipError_t e = hipMemcpyAsync(F.full, f, sizeof(double) * 19 * g.N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_moments_full<T>, fluid_grid(g), b, 0, s, g, F.full, (const T*)F.geo, (T*)F.mom);
  hipLaunchKernelGGL(k_hist_full<T>, fluid_grid(g), b, 0, s, g, F.full, (const T*)F.geo, (const T*)F.mom,
                     (const T*)F.uw, F.moving[0], F.moving[1], (const T*)F.up, tau, (T*)F.hist[F.cur]);
  hipLaunchKernelGGL(k_full_to_streamed<T>, fluid_grid(g), b, 0, s, g, F.full, (const T*)F.hist[F.cur],
                     (const T*)F.geo);
  hipLaunchKernelGGL(k_unpull<T>, fluid_grid(g), b, 0, s, g, (const double*)F.full, (T*)F.pop[F.cur]);
  return hipGetLastError();
}

template <class T> hipError_t launch_get_pops(Fields& F, hipStream_t s, double* out) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_get_pops<T>, fluid_grid(F.g), b, 0, s, F.g, (const T*)F.pop[F.cur], (const T*)F.hist[F.cur],
                     (const T*)F.geo, (const T*)F.vin, out);
  return hipGetLastError();
}

template <class T> hipError_t launch_get_hist(Fields& F, hipStream_t s, double* out) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_get_hist<T>, fluid_grid(F.g), b, 0, s, F.g, (const T*)F.hist[F.cur], out);
  return hipGetLastError();
}

template <class T> hipError_t launch_get_geo(Fields& F, hipStream_t s, double* out) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_get_geo<T>, fluid_grid(F.g), b, 0, s, F.g, (const T*)F.geo, out);
  return hipGetLastError();
}

template <class T> hipError_t launch_moments_out(Fields& F, hipStream_t s, double* rho, double* u, int cart) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_moments_out<T>, fluid_grid(F.g), b, 0, s, F.g, (const T*)F.pop[F.cur], (const T*)F.hist[F.cur],
                     (const T*)F.geo, (const T*)F.vin, F.jac, rho, u, cart);
  return hipGetLastError();
}

template <class T>
hipError_t launch_wall_force(Fields& F, hipStream_t s, int wall, T tau, double* total, double* per_node, int mem,
                             double* part, unsigned* count) {
  const long long nb = wall_force_blocks(F.g);
  hipLaunchKernelGGL(k_wall_force<T>, dim3((unsigned)nb), dim3(WF_THREADS), 0, s, F.g, wall, mem, (const T*)F.pop[F.cur],
                     (const T*)F.hist[F.cur], (const T*)F.geo, (const T*)F.vin, F.jac, tau, per_node,
                     part ? part : F.part, part ? count : F.count, total);
  return hipGetLastError();
}

#define LBM_INST(T)                                                                                     \
  template hipError_t launch_step<T>(Fields&, hipStream_t, T, hipEvent_t*);                            \
  template hipError_t launch_feq_full<T>(Fields&, hipStream_t, const double*, const double*);          \
  template hipError_t launch_set_state<T>(Fields&, hipStream_t, const double*, T);                     \
  template hipError_t launch_get_pops<T>(Fields&, hipStream_t, double*);                               \
  template hipError_t launch_get_hist<T>(Fields&, hipStream_t, double*);                               \
  template hipError_t launch_get_geo<T>(Fields&, hipStream_t, double*);                                \
  template hipError_t launch_moments_out<T>(Fields&, hipStream_t, double*, double*, int);              \
  template hipError_t launch_wall_force<T>(Fields&, hipStream_t, int, T, double*, double*, int, double*,   \
                                           unsigned*);
LBM_INST(double)
LBM_INST(float)
#undef LBM_INST
template hipError_t launch_wall_force_noalloc<double>(Fields&, hipStream_t, int, double, double*, double*, int,
                                                      void*);
template hipError_t launch_wall_force_noalloc<float>(Fields&, hipStream_t, int, float, double*, double*, int,
                                                     void*);

}  // namespace lbm
