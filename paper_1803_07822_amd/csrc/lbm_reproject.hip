// Re-projection of the state onto a new chart (Sec. IV.B).
//
// The populations depend on space only through their Hermite moments, so the
// state is carried by its moments: rho, rho u and the momentum flux
// Pi = sqrt g sum f c c at the old nodes, and the forcing history (A, B, C).
// They are pushed to Cartesian components with the old J (tensor rule,
// Eq. vector_transform), interpolated trilinearly at psi(x~) = h^{-1}(h~(x~))
// (found by Newton on the trilinear interpolant of the old chart), pulled
// back with the new J^{-1}, and recomposed to second order in the new chart
// (a2 = Pi~ - c_s^2 rho I).  The layers outside the walls carry ghosts: rho u
// by the mirror rule about rho v_wall, the other moments by linear
// extrapolation.  Moments and geometry are handled in FP64; populations end in
// the storage precision.
#include <climits>

#include "lbm_internal.h"
#include "lbm_pull.h"

namespace lbm {

namespace {

// a mod n for any a; the common case (within one period) without a division.
__device__ __forceinline__ int wrapr(int a, int n) {
  if (a >= 0 && a < n) return a;
  if (a < 0 && a >= -n) return a + n;
  if (a >= n && a < 2 * n) return a - n;
  a %= n;
  return a < 0 ? a + n : a;
}

// The 8 corners of the trilinear cell with base (bx, by, bz) in a periodic
// (x, z) grid of `layers` y-layers (row y stored at y + yoff), and the
// fractional position in the cell.
struct Cell {
  unsigned e[8];  // element offsets (grids stay below 2^32 elements per field)
  double fr[3];
};

__device__ __forceinline__ void cell_setup(const Grid& g, int layers, int yoff, int bx, int by, int bz,
                                           const double fr[3], Cell& c) {
  const int x0 = wrapr(bx, g.nx), x1 = wrapr(bx + 1, g.nx);
  const int z0 = wrapr(bz, g.nz), z1 = wrapr(bz + 1, g.nz);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ox = q & 1, oy = (q >> 1) & 1, oz = (q >> 2) & 1;
    c.e[q] = ((unsigned)(oz ? z1 : z0) * layers + (unsigned)(by + oy + yoff)) * (unsigned)g.nx + (ox ? x1 : x0);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) c.fr[a] = fr[a];
}

// A cell whose layers by, by + 1 are the two fluid rows on either side of the
// plate, in a column pair touching a plate column, is moved to the side of the
// node being built (side 0 below, 1 above): the fields are then extrapolated
// linearly from that side instead of mixed across the plate.  The position
// search and the moment interpolation of a node use the same rule.
__device__ __forceinline__ int plate_side_layer(const Grid& g, int side, int bx, int by) {
  if (!g.pj || by != g.pj) return by;
  const int c0 = wrapr(bx, g.nx), c1 = wrapr(bx + 1, g.nx);
  if ((c0 >= g.pi0 && c0 <= g.pi1) || (c1 >= g.pi0 && c1 <= g.pi1)) return side ? g.pj + 1 : g.pj - 1;
  return by;
}

// Trilinear value from the eight corner values of a cell (corner q at offsets
// (q & 1, (q >> 1) & 1, (q >> 2) & 1)) and its gradient in cell coordinates.
__device__ __forceinline__ double trilin_corners(const double F[8], const double fr[3], double grad[3]) {
  double v = 0.0;
  grad[0] = grad[1] = grad[2] = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ox = q & 1, oy = (q >> 1) & 1, oz = (q >> 2) & 1;
    const double wx = ox ? fr[0] : 1.0 - fr[0];
    const double wy = oy ? fr[1] : 1.0 - fr[1];
    const double wz = oz ? fr[2] : 1.0 - fr[2];
    v += wx * wy * wz * F[q];
    grad[0] += (ox ? 1.0 : -1.0) * wy * wz * F[q];
    grad[1] += wx * (oy ? 1.0 : -1.0) * wz * F[q];
    grad[2] += wx * wy * (oz ? 1.0 : -1.0) * F[q];
  }
  return v;
}

// Newton step size at which psi counts as found, relative to the position:
// far below the interpolation's own rounding in each storage precision.
template <class T> constexpr double NEWTON_TOL = sizeof(T) == 4 ? 1e-10 : 1e-13;

constexpr int NMF = 20;  // 0 rho, 1-3 j, 4-9 Pi, 10 A, 11-13 B, 14-19 C (Cartesian)

// The moment fields are stored node by node ([node][20]): the 20 values of a
// node are 80 (FP32) or 160 (FP64) contiguous bytes, moved with 16-byte
// vector loads and stores, which the interpolation's eight corner gathers
// per node need most.
template <class T> struct MfVec;
template <> struct MfVec<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <> struct MfVec<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};

template <class T> __device__ __forceinline__ void mf_load(const T* __restrict__ mf, long long e, double out[NMF]) {
  typedef typename MfVec<T>::v V;
  constexpr int W = MfVec<T>::W;
  const V* p = (const V*)(mf + e * NMF);
#pragma unroll
  for (int q = 0; q < NMF / W; ++q) {
    const V v = p[q];
#pragma unroll
    for (int r = 0; r < W; ++r) out[q * W + r] = (double)v[r];
  }
}

template <class T> __device__ __forceinline__ void mf_store(T* __restrict__ mf, long long e, const double in[NMF]) {
  typedef typename MfVec<T>::v V;
  constexpr int W = MfVec<T>::W;
  V* p = (V*)(mf + e * NMF);
#pragma unroll
  for (int q = 0; q < NMF / W; ++q) {
    V v;
#pragma unroll
    for (int r = 0; r < W; ++r) v[r] = (T)in[q * W + r];
    p[q] = v;
  }
}

// The moment fields are stored in the state's precision as deviations from
// the state at rest (rho = 1, Pi = I/3 in Cartesian components), so that FP32
// keeps their small variations; every operation on them (ghost layers,
// interpolation) is linear, and the rest values are added back in FP64.
__device__ __forceinline__ double mf_rest(int q) {
  return q == 0 ? 1.0 : ((q == 4 || q == 7 || q == 9) ? 1.0 / 3.0 : 0.0);
}

__device__ __forceinline__ void inv3d(const double m[3][3], double r[3][3]) {
  const double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                     m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                     m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
  const double idet = 1.0 / det;
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) * idet;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * idet;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * idet;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) * idet;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * idet;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * idet;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) * idet;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * idet;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * idet;
}

// Cartesian moment fields at the old fluid nodes (Y: the old chart moves the
// nodes along y only).
template <class T, bool Y>
__global__ __launch_bounds__(BX * BY) void k_rp_moments(Grid g, const T* __restrict__ pop, const T* __restrict__ hist, const T* __restrict__ geo,
                             const T* __restrict__ vin, const double* __restrict__ jac, T* __restrict__ mf) {
  int i, jf, k;
  if (!xcd_fluid_node(g, i, jf, k)) return;
  const long long n = ((long long)k * g.H + jf) * g.nx + i;
  const long long e = ((long long)k * g.ny + (jf + 1)) * g.nx + i;
  // J is loaded first, so that its round trip overlaps the pulls'
  double J[3][3];
  jac_at<Y>(jac, g.N, n, J);
  Coef<T> c;
  c.A = hist[H_A * g.N + n];
#pragma unroll
  for (int a = 0; a < 3; ++a) c.B[a] = hist[(H_B + a) * g.N + n];
#pragma unroll
  for (int q = 0; q < 6; ++q) c.C[q] = hist[(H_C + q) * g.N + n];
  const T sgd = geo[G_SG * g.N + n];
  const T isg = T(1) / (T(1) + sgd);
  T Fp[Q], gv[Q];
  forcing_pops(c, isg, Fp);
  pull_all(pop, hist, geo, vin, g, pos_at(g, i, jf, k), gv);
  double s = 0, jv[3] = {0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const double v = (double)gv[l] + 0.5 * (double)Fp[l];
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    s += v;
    if (x) jv[0] += x * v;
    if (y) jv[1] += y * v;
    if (z) jv[2] += z * v;
    if (x) P[0] += v;
    if (y) P[3] += v;
    if (z) P[5] += v;
    if (x && y) P[1] += x * y * v;
    if (x && z) P[2] += x * z * v;
    if (y && z) P[4] += y * z * v;
  });
  const double sg = 1.0 + (double)sgd;
  // f = w + f~: sum w = 1, sum w c c = I/3
  const double rho = sg * (1.0 + s);
  double j[3], Pm[3][3], Bv[3], Cm[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    j[a] = sg * jv[a];
    Bv[a] = (double)c.B[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Pm[a][b] = sg * ((a == b ? 1.0 / 3.0 : 0.0) + P[sym(a, b)]);
      Cm[a][b] = (double)c.C[sym(a, b)];
    }
  double out[NMF];
  out[0] = rho - mf_rest(0);
  out[10] = (double)c.A;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out[1 + a] = J[a][0] * j[0] + J[a][1] * j[1] + J[a][2] * j[2];
    out[11 + a] = J[a][0] * Bv[0] + J[a][1] * Bv[1] + J[a][2] * Bv[2];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      double sp = 0.0, sc = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          sp += J[a][p] * Pm[p][r] * J[b][r];
          sc += J[a][p] * Cm[p][r] * J[b][r];
        }
      out[4 + sym(a, b)] = sp - mf_rest(4 + sym(a, b));
      out[14 + sym(a, b)] = sc;
    }
  mf_store(mf, e, out);
}

// Wall-layer ghosts of the moment fields: linear extrapolation from the two
// nearest fluid layers; rho u by the mirror rule about rho v_wall instead.
template <class T>
__global__ __launch_bounds__(BX * BY) void k_rp_ghost(Grid g, const double* __restrict__ vwall, T* __restrict__ mf) {
  const int i = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  for (int w = 0; w < 2; ++w) {
    const int jg = w == 0 ? 0 : g.ny - 1, jm = w == 0 ? 1 : g.ny - 2, jm2 = w == 0 ? 2 : g.ny - 3;
    const long long eg = ((long long)k * g.ny + jg) * g.nx + i;
    const long long em = ((long long)k * g.ny + jm) * g.nx + i;
    const long long em2 = ((long long)k * g.ny + jm2) * g.nx + i;
    double m1[NMF], m2[NMF], gv[NMF];
    mf_load(mf, em, m1);
    mf_load(mf, em2, m2);
#pragma unroll
    for (int q = 0; q < NMF; ++q) gv[q] = 2.0 * m1[q] - m2[q];
    const long long c = (((long long)w * g.nz + k) * g.nx + i) * 3;
    const double rho_m = mf_rest(0) + m1[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) gv[1 + a] = 2.0 * rho_m * vwall[c + a] - m1[1 + a];
    mf_store(mf, eg, gv);
  }
}

// New state at the new fluid nodes: the streamed deviations g~ written
// straight into the pull layout, and the new history (storage precision).
// Y: the old and the new chart both move the nodes along y only, so psi keeps
// the node's x and z, its search is one-dimensional, and two rows of the new J
// are exact.
template <class T, bool Y>
__global__ __launch_bounds__(BX * BY) void k_rp_new(Grid g, const double* __restrict__ chart, const double* __restrict__ uold,
                         const T* __restrict__ mf, const double* __restrict__ jac, const T* __restrict__ geo,
                         T* __restrict__ pop, T* __restrict__ hist) {
  int i, jf, k;
  if (!xcd_fluid_node(g, i, jf, k)) return;
  const long long n = ((long long)k * g.H + jf) * g.nx + i;
  const long long NC = (long long)g.nz * g.ny * g.nx, NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const long long pc = ((long long)k * g.ny + (jf + 1)) * g.nx + i;
  // read before the search, so that its latency is not a phase of its own
  const T sgd = geo[G_SG * g.N + n];
  // psi: xi + u_old(xi) = p.  Start from one fixed-point step off the node,
  // xi = p - u_old(node), which lands in the cell of the solution unless the
  // chart moved by most of a cell; the corners of the old displacement are
  // gathered once per cell and reused by the Newton iterations in it.
  const int side = jf >= g.pj ? 1 : 0;
  const long long e0 = ((long long)k * (g.ny + 6) + (jf + 1 + 3)) * g.nx + i;
  double xi[3];
  // the new J (Y: its varying row), read before the search for the same reason
  double J[3][3];
  jac_at<Y>(jac, g.N, n, J);
  if constexpr (Y) {
    // x and z displacements are zero in both charts: xi = (i, y, k) with
    // y + u_old,y(i, y, k) = p_y, linear between the two layers around y.
    // The node's own layer and the two beside it are loaded together: the
    // walls move much less than a layer per update, so the first cell is
    // one of the two they span and its corners need no second round trip.
    const double py = chart[NC + pc];
    const double* uy = uold + NE;
    const long long col = (long long)k * (g.ny + 6) * g.nx + i;
    const int jn = jf + 1;  // the node's layer
    const double Um = uy[e0 - g.nx], Uc = uy[e0], Up = uy[e0 + g.nx];
    xi[0] = (double)i;
    xi[2] = (double)k;
    xi[1] = py - Uc;
    int cby = INT_MIN;
    double U0 = 0.0, U1 = 0.0;
    for (int it = 0; it < 50; ++it) {
      int by = (int)floor(xi[1]);
      if (by < -3) by = -3;
      if (by > g.ny + 1) by = g.ny + 1;
      by = plate_side_layer(g, side, i, by);
      if (by != cby) {
        if (by == jn - 1) {
          U0 = Um;
          U1 = Uc;
        } else if (by == jn) {
          U0 = Uc;
          U1 = Up;
        } else {
          U0 = uy[col + (long long)(by + 3) * g.nx];
          U1 = uy[col + (long long)(by + 4) * g.nx];
        }
        cby = by;
      }
      const double fr = xi[1] - by;
      const double r = xi[1] + ((1.0 - fr) * U0 + fr * U1) - py;
      const double d = r / (1.0 + (U1 - U0));
      xi[1] -= d;
      if (fabs(d) <= NEWTON_TOL<T> * (1.0 + xi[0] + fabs(xi[1]) + xi[2])) break;
    }
  } else {
    const double p[3] = {chart[pc], chart[NC + pc], chart[2 * NC + pc]};
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = p[a] - uold[a * NE + e0];
    int cbx = INT_MIN, cby = INT_MIN, cbz = INT_MIN;
    double U[3][8];
    for (int it = 0; it < 50; ++it) {
      double r[3], Jm[3][3], Ji[3][3];
      // cell of the extended grid (layers -3 .. ny+2) holding xi
      const int bx = (int)floor(xi[0]), bz = (int)floor(xi[2]);
      int by = (int)floor(xi[1]);
      if (by < -3) by = -3;
      if (by > g.ny + 1) by = g.ny + 1;
      by = plate_side_layer(g, side, bx, by);
      if (bx != cbx || by != cby || bz != cbz) {
        Cell c;
        const double fr0[3] = {0.0, 0.0, 0.0};
        cell_setup(g, g.ny + 6, 3, bx, by, bz, fr0, c);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int q = 0; q < 8; ++q) U[a][q] = uold[a * NE + c.e[q]];
        cbx = bx;
        cby = by;
        cbz = bz;
      }
      const double fr[3] = {xi[0] - bx, xi[1] - by, xi[2] - bz};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double gr[3];
        r[a] = xi[a] + trilin_corners(U[a], fr, gr) - p[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) Jm[a][b] = (a == b ? 1.0 : 0.0) + gr[b];
      }
      inv3d(Jm, Ji);
      double dmax = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double d = Ji[a][0] * r[0] + Ji[a][1] * r[1] + Ji[a][2] * r[2];
        xi[a] -= d;
        dmax = fmax(dmax, fabs(d));
      }
      if (dmax <= NEWTON_TOL<T> * (1.0 + fabs(xi[0]) + fabs(xi[1]) + fabs(xi[2]))) break;
    }
  }
  // trilinear interpolation of the moment fields, y inside layers 0..ny-1
  double q1 = xi[1];
  if (q1 < 0.0) q1 = 0.0;
  if (q1 > g.ny - 1.0) q1 = g.ny - 1.0;
  const int bx = (int)floor(xi[0]), bz = (int)floor(xi[2]);
  int by = (int)floor(q1);
  if (by > g.ny - 2) by = g.ny - 2;
  if (by < 0) by = 0;
  by = plate_side_layer(g, side, bx, by);
  const double fr[3] = {xi[0] - bx, q1 - by, xi[2] - bz};
  Cell cl;
  cell_setup(g, g.ny, 0, bx, by, bz, fr, cl);
  double m[NMF];
#pragma unroll
  for (int q = 0; q < NMF; ++q) m[q] = 0.0;
  auto corner = [&](auto C) {
    constexpr int c = decltype(C)::value;
    constexpr int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
    const double w = (ox ? fr[0] : 1.0 - fr[0]) * (oy ? fr[1] : 1.0 - fr[1]) * (oz ? fr[2] : 1.0 - fr[2]);
    double mc[NMF];
    mf_load(mf, cl.e[c], mc);
#pragma unroll
    for (int q = 0; q < NMF; ++q) m[q] += w * mc[q];
  };
  // A chart that moves the nodes along y only (a wall displaced along its
  // normal) leaves psi on the node's own x and z, so the corners at x + 1 and
  // z + 1 weigh exactly zero and adding them changes no bit of the sum.  The
  // choice is made per wave (no lane diverges): the four-corner-pairs gather
  // runs only when some lane of the wave needs it.
  if (!Y && __any(fr[0] != 0.0 || fr[2] != 0.0)) {
    Unroll<int, 8>::run(corner);
  } else {
    corner(std::integral_constant<int, 0>());
    corner(std::integral_constant<int, 2>());
  }
#pragma unroll
  for (int q = 0; q < NMF; ++q) m[q] += mf_rest(q);
  // pull back with the new J^{-1}
  double Ji[3][3];
  inv3d(J, Ji);
  double Pc[3][3], Cc[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Pc[a][b] = m[4 + sym(a, b)];
      Cc[a][b] = m[14 + sym(a, b)];
    }
  double jt[3], Bt[3], a2[6], Ct[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    jt[a] = Ji[a][0] * m[1] + Ji[a][1] * m[2] + Ji[a][2] * m[3];
    Bt[a] = Ji[a][0] * m[11] + Ji[a][1] * m[12] + Ji[a][2] * m[13];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      double sp = 0.0, sc = 0.0;
#pragma unroll
      for (int p1 = 0; p1 < 3; ++p1)
#pragma unroll
        for (int r1 = 0; r1 < 3; ++r1) {
          sp += Ji[a][p1] * Pc[p1][r1] * Ji[b][r1];
          sc += Ji[a][p1] * Cc[p1][r1] * Ji[b][r1];
        }
      a2[sym(a, b)] = sp - (a == b ? m[0] / 3.0 : 0.0);
      Ct[sym(a, b)] = sc;
    }
  // new history (in storage precision) and the F(t-1)/2 it implies
  Coef<T> c;
  c.A = (T)m[10];
#pragma unroll
  for (int a = 0; a < 3; ++a) c.B[a] = (T)Bt[a];
#pragma unroll
  for (int q = 0; q < 6; ++q) c.C[q] = (T)Ct[q];
  hist[H_A * g.N + n] = c.A;
#pragma unroll
  for (int a = 0; a < 3; ++a) hist[(H_B + a) * g.N + n] = c.B[a];
#pragma unroll
  for (int q = 0; q < 6; ++q) hist[(H_C + q) * g.N + n] = c.C[q];
  const T isg = T(1) / (T(1) + sgd);
  T Fp[Q];
  forcing_pops(c, isg, Fp);
  // f~ - w = (w/sqrt g)[rho + 3 j.c + 4.5 a2:cc - 1.5 tr a2] - w
  const double sg = 1.0 + (double)sgd;
  const double a0 = m[0] - sg;  // (rho/sqrt g - 1) sqrt g
  // Store g~_l = f~_l - F_l/2 in the pull layout: at x - c_l when the link
  // from there is open, else (a link through a wall or the plate) in the
  // bounce-back slot opp(l) of this node.  Every slot of the layout has
  // exactly one writer.  The store takes a selected address, not a branch.
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    const double fdev = wgt(l) / sg * hermite_term<double, l>(a0, jt, a2);
    const T v = (T)(fdev - 0.5 * (double)Fp[l]);
    const int js = jf - y;
    const bool cut = js < 0 || js >= g.H || plate_cut(g, i, jf, -x, -y);
    const int is = x ? wrapr(i - x, g.nx) : i;
    const int ks = z ? wrapr(k - z, g.nz) : k;
    const long long dst =
        cut ? (long long)opp(l) * g.N + n : (long long)l * g.N + ((long long)ks * g.H + js) * g.nx + is;
    pop[dst] = v;
  });
}

}  // namespace

// Precondition: F.chart holds the new chart; uext/jac/geo still describe the
// old one.  Computes the new geometry on the way.
template <class T> hipError_t launch_reproject(Fields& F, hipStream_t s, const double Fc[3], T tau) {
  (void)tau;
  const Grid g = F.g;
  dim3 b(BX, BY);
  // the moments are pushed to Cartesian components with the old chart's J
  auto* km = F.uext_yonly[F.uext_cur] ? k_rp_moments<T, true> : k_rp_moments<T, false>;
  hipLaunchKernelGGL(km, xcd_fluid_grid(g), b, 0, s, g, (const T*)F.pop[F.cur], (const T*)F.hist[F.cur],
                     (const T*)F.geo, (const T*)F.vin, (const double*)F.jac, (T*)F.mf);
  hipLaunchKernelGGL(k_rp_ghost<T>, col_grid(g), b, 0, s, g, (const double*)F.vwall, (T*)F.mf);
  const int old = F.uext_cur;
  F.uext_cur ^= 1;
  hipError_t e = launch_geometry<T>(F, s, Fc);
  if (e != hipSuccess) return e;
  auto* kn = F.chart_yonly && F.uext_yonly[old] ? k_rp_new<T, true> : k_rp_new<T, false>;
  hipLaunchKernelGGL(kn, xcd_fluid_grid(g), b, 0, s, g, (const double*)F.chart, (const double*)F.uext[old],
                     (const T*)F.mf, (const double*)F.jac, (const T*)F.geo, (T*)F.pop[F.cur],
                     (T*)F.hist[F.cur]);
  return hipGetLastError();
}

template hipError_t launch_reproject<double>(Fields&, hipStream_t, const double*, double);
template hipError_t launch_reproject<float>(Fields&, hipStream_t, const double*, float);

}  // namespace lbm
