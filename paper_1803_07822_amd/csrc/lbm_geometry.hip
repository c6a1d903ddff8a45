// Geometry precompute (FP64): chart -> J, g, g^{-1}, sqrt g, Christoffel
// symbols and the contravariant body force at every fluid node (App. A), with
// the fourth-order isotropic lattice derivative of App. D,
//   D_i f = G_i[f - (c_s^2/2) L f],
//   G_i f = (1/c_s^2) sum_l w_l c_l^i f(x + c_l),
//   L f   = (2/c_s^2) sum_l w_l (f(x + c_l) - f(x)).
// The chart is split into the identity and a displacement u that is periodic
// in x and z (the stencils are exact on the identity, so J = I + D u).  In y,
// u is continued three layers past each wall layer by the cubic through the
// four nearest layers.  Each stage is a separate, embarrassingly parallel
// pass over the y-extended grid (memory bound; runs once per metric update).
#include "lbm_internal.h"

namespace lbm {

namespace {

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// extended-grid index, layer j in [-3, ny+2]
__device__ __forceinline__ long long eidx(const Grid& g, int i, int j, int k) {
  return ((long long)k * (g.ny + 6) + (j + 3)) * g.nx + i;
}

__device__ __forceinline__ void inv3(const double m[3][3], double r[3][3], double& det) {
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

// Shape of the plate's displacement across the channel (Sec. IV.A.1 (ii)):
// the natural cubic spline through (0, 0), (eta_p, 1), (H, 0) in the
// wall-normal coordinate eta (zero second derivative at both walls).  On each
// piece it is the cubic with the end values and the end second derivatives
// 0 (at the wall) and M (at the plate); matching the slopes at the plate
// gives M = -3 (1/a + 1/b) / H for the knot spacings a = eta_p, b = H - eta_p.
__device__ __forceinline__ double plate_spline(double eta, int eta_p, int H) {
  const double a = eta_p, b = H - eta_p, M = -3.0 * (1.0 / a + 1.0 / b) / H;
  const double len = eta <= a ? a : b;
  const double t = eta <= a ? eta : H - eta;  // distance from the nearer wall's knot
  return t * (M * t * t + 6.0 - M * len * len) / (6.0 * len);
}

// Chart of the walls and the plate: the wall displacements blended linearly
// across the channel (Sec. IV.A.1 (i)) plus the plate's cross-section
// displacement carried by plate_spline; eta = xi_y - 1/2 puts the halfway
// walls at 0 and H and the plate (between fluid rows pj - 1 and pj) at pj.
// XZ: write the x and z components (i, k); they are left in place when the
// chart already holds them from an earlier call.  A new displacement of one
// field (which: 0 bottom wall, 1 top wall, 2 plate; -1 none) comes from src
// (NULL: zero) and is stored into the context's copy by the layer-0 thread of
// each column, in place of a separate copy.
template <bool XZ>
__global__ __launch_bounds__(BX * BY) void k_chart_from_disp(Grid g, double* __restrict__ disp,
                                                             double* __restrict__ dplate,
                                                             double* __restrict__ chart, int which,
                                                             const double* __restrict__ src) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const long long NC = (long long)g.nz * g.ny * g.nx, ncol = (long long)g.nz * g.nx;
  const long long p = ((long long)k * g.ny + j) * g.nx + i;
  const long long q = (long long)k * g.nx + i;
  const double vin = which >= 0 && src ? src[q] : 0.0;
  const double d0 = which == 0 ? vin : disp[q], d1 = which == 1 ? vin : disp[ncol + q];
  if (which >= 0 && j == 0) (which == 2 ? dplate : disp + which * ncol)[q] = vin;
  const double eta = j - 0.5, s = eta / g.H;
  double y = (double)j + (1.0 - s) * d0 + s * d1;
  if (g.pj) y += (which == 2 ? vin : dplate[q]) * plate_spline(eta, g.pj, g.H);
  chart[NC + p] = y;
  if (XZ) {
    chart[p] = (double)i;
    chart[2 * NC + p] = (double)k;
  }
}

// u = chart - xi on layers 0..ny-1, cubic continuation on -3..-1 and ny..ny+2.
// Y: the chart moves the nodes along y only, so u_x = u_z = 0 exactly; XZ:
// write those two components (Y: zeros), else they are already in place.
template <bool Y, bool XZ>
__global__ __launch_bounds__(BX * BY) void k_uext(Grid g, const double* __restrict__ chart, double* __restrict__ u) {
  const int i = blockIdx.x * BX + threadIdx.x, je = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || je >= g.ny + 6) return;
  const int j = je - 3;
  const long long NC = (long long)g.nz * g.ny * g.nx, NE = (long long)g.nz * (g.ny + 6) * g.nx;
  auto uat = [&](int a, int jj) {
    const double xi = a == 0 ? (double)i : (a == 1 ? (double)jj : (double)k);
    return chart[a * NC + ((long long)k * g.ny + jj) * g.nx + i] - xi;
  };
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a != 1 && !XZ) continue;
    if (Y && a != 1) {
      u[a * NE + eidx(g, i, j, k)] = 0.0;
      continue;
    }
    double v;
    if (j >= 0 && j < g.ny) {
      v = uat(a, j);
    } else {
      // Lagrange cubic through the four nearest layers, evaluated 1..3 layers out
      const int d = j < 0 ? -j : j - (g.ny - 1);  // 1, 2, 3
      const int b0 = j < 0 ? 0 : g.ny - 1, s = j < 0 ? 1 : -1;
      const double u0 = uat(a, b0), u1 = uat(a, b0 + s), u2 = uat(a, b0 + 2 * s), u3 = uat(a, b0 + 3 * s);
      if (d == 1)
        v = 4.0 * u0 - 6.0 * u1 + 4.0 * u2 - u3;
      else if (d == 2)
        v = 10.0 * u0 - 20.0 * u1 + 15.0 * u2 - 4.0 * u3;
      else
        v = 20.0 * u0 - 45.0 * u1 + 36.0 * u2 - 10.0 * u3;
    }
    u[a * NE + eidx(g, i, j, k)] = v;
  }
}

// ------------------------------------------------ plane-marching stencils
// The three stencil passes of the precompute (smoothing, J and g, the metric
// derivatives with the fluid-node geometry) read the 18 lattice neighbours
// of every node.  A block owns a 64 x 4 tile of (x, layer) and marches along a
// chunk of z-planes; the input components of three consecutive planes of the
// tile plus a one-node halo sit in an LDS ring, so each input value is read
// from memory about once per pass.
constexpr int MX = BX + 2, MY = BY + 2, MN = MX * MY;
constexpr int MZC = 16;  // planes per block

struct March {
  int i0, j0, z0, z1;  // tile origin (x, layer) and z range
  int tx, ty;          // thread position in the tile
};

__device__ __forceinline__ bool march_setup(const Grid& g, int jlo, int jhi, March& m) {
  m.i0 = blockIdx.x * BX;
  m.j0 = jlo + blockIdx.y * BY;
  m.z0 = blockIdx.z * MZC;
  m.z1 = min(m.z0 + MZC, g.nz);
  m.tx = threadIdx.x;
  m.ty = threadIdx.y;
  return m.j0 <= jhi;  // uniform per block
}

// Plane k (wrapped) of NC components into one ring slot; layers outside the
// extended grid are never read by an output inside [jlo, jhi].  Each thread
// loads its (at most MPT) entries before writing any of them, and an entry
// outside the grid reads a valid dummy address instead of branching, so the
// loads of a plane are all in flight together.
constexpr int MPT = (MN + BX * BY - 1) / (BX * BY);
template <int NC>
__device__ __forceinline__ void march_load(const Grid& g, const March& m, int k, const double* __restrict__ in,
                                           double (*slot)[MN]) {
  k = wrap(k, g.nz);
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  double v[MPT][NC];
  bool ok[MPT];
#pragma unroll
  for (int r = 0; r < MPT; ++r) {
    const int e = m.ty * BX + m.tx + r * BX * BY;
    const int hx = e % MX, hy = e / MX;
    const int i = wrap(m.i0 - 1 + hx, g.nx), j = m.j0 - 1 + hy;
    ok[r] = e < MN && !(m.i0 - 1 + hx > g.nx || j < -3 || j > g.ny + 2);
    const long long p = ok[r] ? eidx(g, i, j, k) : 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[r][c] = in[c * NE + p];
  }
#pragma unroll
  for (int r = 0; r < MPT; ++r)
    if (ok[r]) {
      const int e = m.ty * BX + m.tx + r * BX * BY;
#pragma unroll
      for (int c = 0; c < NC; ++c) slot[c][e] = v[r][c];
    }
}

// Ring of four plane slots: the load of plane k+1 overwrites plane k-3, whose
// last reader (the stencil of plane k-2) every thread has finished before
// the barrier of the previous plane, so one barrier per plane suffices.
__device__ __forceinline__ int rs(int k) { return (k + 4) & 3; }

// G_i f = 3 sum_l w_l c_l^i f(x + c_l) of component c at the tile node, from
// the ring (planes k-1, k, k+1 in slots sm, s0, sp).
template <int NC>
__device__ __forceinline__ void march_grad(const double (*sm)[MN], const double (*s0)[MN], const double (*sp)[MN],
                                           int e0, int c, double d[3]) {
  double s0x = 0, s1 = 0, s2 = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    if (l == 0) return;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    const double(*sl)[MN] = z < 0 ? sm : (z > 0 ? sp : s0);
    const double fv = sl[c][e0 + y * MX + x];
    if (x) s0x += wgt(l) * x * fv;
    if (y) s1 += wgt(l) * y * fv;
    if (z) s2 += wgt(l) * z * fv;
  });
  d[0] = 3.0 * s0x;
  d[1] = 3.0 * s1;
  d[2] = 3.0 * s2;
}

// out = in - (c_s^2/2) L in = in - sum_l w_l (in(x+c_l) - in(x)) on layers [jlo, jhi]
template <int NC>
__global__ __launch_bounds__(BX * BY) void k_smooth(Grid g, int jlo, int jhi, const double* __restrict__ in,
                                                    double* __restrict__ out) {
  __shared__ double ring[4][NC][MN];
  March m;
  if (!march_setup(g, jlo, jhi, m)) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const int i = m.i0 + m.tx, j = m.j0 + m.ty;
  const bool act = i < g.nx && j <= jhi;
  const int e0 = (m.ty + 1) * MX + (m.tx + 1);
  march_load<NC>(g, m, m.z0 - 1, in, ring[rs(m.z0 - 1)]);
  march_load<NC>(g, m, m.z0, in, ring[rs(m.z0)]);
  for (int k = m.z0; k < m.z1; ++k) {
    march_load<NC>(g, m, k + 1, in, ring[rs(k + 1)]);
    __syncthreads();
    if (act) {
      const double(*sm)[MN] = ring[rs(k - 1)];
      const double(*s0)[MN] = ring[rs(k)];
      const double(*sp)[MN] = ring[rs(k + 1)];
      const long long p = eidx(g, i, j, k);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double f0 = s0[c][e0];
        double s = 0.0;
        for_q([&](auto L) {
          constexpr int l = decltype(L)::value;
          if (l == 0) return;
          constexpr int x = cx(l), y = cy(l), z = cz(l);
          const double(*sl)[MN] = z < 0 ? sm : (z > 0 ? sp : s0);
          s += wgt(l) * (sl[c][e0 + y * MX + x] - f0);
        });
        out[c * NE + p] = f0 - s;
      }
    }
  }
}

// The smoothing above applied to g = J^T J of a chart that moves the nodes
// along y only, g formed at every stencil point from the varying row of J
// (three components read instead of six).
__global__ __launch_bounds__(BX * BY) void k_smooth_gy(Grid g, int jlo, int jhi, const double* __restrict__ row,
                                                       double* __restrict__ out) {
  __shared__ double ring[4][3][MN];
  March m;
  if (!march_setup(g, jlo, jhi, m)) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const int i = m.i0 + m.tx, j = m.j0 + m.ty;
  const bool act = i < g.nx && j <= jhi;
  const int e0 = (m.ty + 1) * MX + (m.tx + 1);
  march_load<3>(g, m, m.z0 - 1, row, ring[rs(m.z0 - 1)]);
  march_load<3>(g, m, m.z0, row, ring[rs(m.z0)]);
  for (int k = m.z0; k < m.z1; ++k) {
    march_load<3>(g, m, k + 1, row, ring[rs(k + 1)]);
    __syncthreads();
    if (act) {
      const double(*sm)[MN] = ring[rs(k - 1)];
      const double(*s0)[MN] = ring[rs(k)];
      const double(*sp)[MN] = ring[rs(k + 1)];
      auto metric_at = [&](const double(*sl)[MN], int o, double gq[6]) {
        metric_of_row(sl[0][o], sl[1][o], sl[2][o], gq);
      };
      double g0[6], s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      metric_at(s0, e0, g0);
      for_q([&](auto L) {
        constexpr int l = decltype(L)::value;
        if (l == 0) return;
        constexpr int x = cx(l), y = cy(l), z = cz(l);
        double gl[6];
        metric_at(z < 0 ? sm : (z > 0 ? sp : s0), e0 + y * MX + x, gl);
#pragma unroll
        for (int q = 0; q < 6; ++q) s[q] += wgt(l) * (gl[q] - g0[q]);
      });
      const long long p = eidx(g, i, j, k);
#pragma unroll
      for (int q = 0; q < 6; ++q) out[q * NE + p] = g0[q] - s[q];
    }
  }
}

// J = I + G v and g = J^T J on layers [-1, ny]; J also stored at fluid nodes.
// Y: v moves the nodes along y only; its y component alone is read (v points
// at it), the rows (1, 0, 0), (0, 0, 1) of J are exact, and the varying row
// (J_yx, J_yy, J_yz) is stored in the first three components of gext in place
// of g, which its readers form from it.  RW (Y only): write the exact rows of
// J at the fluid nodes, else they are already in place.
template <bool Y, bool RW>
__global__ __launch_bounds__(BX * BY) void k_jac_metric(Grid g, const double* __restrict__ v,
                                                        double* __restrict__ gext, double* __restrict__ jac) {
  constexpr int NV = Y ? 1 : 3;
  __shared__ double ring[4][NV][MN];
  const int jlo = -1, jhi = g.ny;
  March m;
  if (!march_setup(g, jlo, jhi, m)) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const int i = m.i0 + m.tx, j = m.j0 + m.ty;
  const bool act = i < g.nx && j <= jhi;
  const int e0 = (m.ty + 1) * MX + (m.tx + 1);
  march_load<NV>(g, m, m.z0 - 1, v, ring[rs(m.z0 - 1)]);
  march_load<NV>(g, m, m.z0, v, ring[rs(m.z0)]);
  for (int k = m.z0; k < m.z1; ++k) {
    march_load<NV>(g, m, k + 1, v, ring[rs(k + 1)]);
    __syncthreads();
    if (act) {
      double J[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double d[3] = {0.0, 0.0, 0.0};
        if (!Y || a == 1) march_grad<NV>(ring[rs(k - 1)], ring[rs(k)], ring[rs(k + 1)], e0, Y ? 0 : a, d);
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][b] = (a == b ? 1.0 : 0.0) + d[b];
      }
      const long long e = eidx(g, i, j, k);
      if constexpr (Y) {
#pragma unroll
        for (int b = 0; b < 3; ++b) gext[b * NE + e] = J[1][b];
      } else {
        double gq[6];
        metric_of(J, gq);
#pragma unroll
        for (int q = 0; q < 6; ++q) gext[q * NE + e] = gq[q];
      }
      if (j >= 1 && j <= g.ny - 2) {
        const long long n = ((long long)k * g.H + (j - 1)) * g.nx + i;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b)
            if (!Y || RW || a == 1) jac[(a * 3 + b) * g.N + n] = J[a][b];
      }
    }
  }
}

// Fluid-node geometry: g^{-1}, sqrt g = det J, Gamma^i_jk = 1/2 g^il (D_j g_kl
// + D_k g_jl - D_l g_jk) with D_l g = G_l w, and F^i = (J^{-1} F_cart)^i.
template <class T, bool Y>
__global__ __launch_bounds__(BX * BY) void k_geo(Grid g, const double* __restrict__ w, const double* __restrict__ gext,
                                                 const double* __restrict__ jac, double F0, double F1, double F2,
                                                 T* __restrict__ geo) {
  __shared__ double ring[4][6][MN];
  const int jlo = 1, jhi = g.ny - 2;
  March m;
  if (!march_setup(g, jlo, jhi, m)) return;
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx;
  const int i = m.i0 + m.tx, j = m.j0 + m.ty;
  const bool act = i < g.nx && j <= jhi;
  const int e0 = (m.ty + 1) * MX + (m.tx + 1);
  march_load<6>(g, m, m.z0 - 1, w, ring[rs(m.z0 - 1)]);
  march_load<6>(g, m, m.z0, w, ring[rs(m.z0)]);
  for (int k = m.z0; k < m.z1; ++k) {
    // this plane's J (and g) are loaded ahead of the ring's next plane and
    // the barrier, so that their round trip overlaps those
    const long long n = ((long long)k * g.H + (j - 1)) * g.nx + i;
    double gm[3][3], J[3][3];
    if (act) {
      jac_at<Y>(jac, g.N, n, J);
      if constexpr (!Y) {
        const long long e = eidx(g, i, j, k);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) gm[a][b] = gext[sym(a, b) * NE + e];
      }
    }
    march_load<6>(g, m, k + 1, w, ring[rs(k + 1)]);
    __syncthreads();
    if (act) {
      double gi[3][3], Ji[3][3], det, detJ;
      if constexpr (Y) {
        double gq[6];
        metric_of_row(J[1][0], J[1][1], J[1][2], gq);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) gm[a][b] = gq[sym(a, b)];
      }
      inv3(gm, gi, det);
      inv3(J, Ji, detJ);
      // dg[l][q] = D_l g_q
      double dg[3][6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        double d[3];
        march_grad<6>(ring[rs(k - 1)], ring[rs(k)], ring[rs(k + 1)], e0, q, d);
        dg[0][q] = d[0];
        dg[1][q] = d[1];
        dg[2][q] = d[2];
      }
      geo[G_SG * g.N + n] = (T)(detJ - 1.0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) geo[(G_GI + sym(a, b)) * g.N + n] = (T)(gi[a][b] - (a == b ? 1.0 : 0.0));
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
          for (int kk = jj; kk < 3; ++kk) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l)
              s += gi[ii][l] * (dg[jj][sym(kk, l)] + dg[kk][sym(jj, l)] - dg[l][sym(jj, kk)]);
            geo[(G_GAM + ii * 6 + sym(jj, kk)) * g.N + n] = (T)(0.5 * s);
          }
      const double Fc[3] = {F0, F1, F2};
#pragma unroll
      for (int a = 0; a < 3; ++a)
        geo[(G_F + a) * g.N + n] = (T)(Ji[a][0] * Fc[0] + Ji[a][1] * Fc[1] + Ji[a][2] * Fc[2]);
    }
  }
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_body_force(Grid g, const double* __restrict__ jac, double F0, double F1, double F2, T* __restrict__ geo) {
  const int i = blockIdx.x * BX + threadIdx.x, jf = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || jf >= g.H) return;
  const long long n = ((long long)k * g.H + jf) * g.nx + i;
  double J[3][3], Ji[3][3], det;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + n];
  inv3(J, Ji, det);
  const double Fc[3] = {F0, F1, F2};
#pragma unroll
  for (int a = 0; a < 3; ++a) geo[(G_F + a) * g.N + n] = (T)(Ji[a][0] * Fc[0] + Ji[a][1] * Fc[1] + Ji[a][2] * Fc[2]);
}

// Chart components J^{-1} v of the Cartesian wall velocity at the fluid node
// next to each wall.
template <class T>
__global__ __launch_bounds__(BX * BY) void k_wall_velocity(Grid g, const double* __restrict__ jac, double* __restrict__ vwall,
                                                           T* __restrict__ uw, int which, const double* __restrict__ src) {
  const int i = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  // a new Cartesian velocity of wall `which` (-1: none) comes from src (NULL:
  // zero) and is stored into the context's copy, in place of a separate copy
  if (which >= 0) {
    const long long c = (((long long)which * g.nz + k) * g.nx + i) * 3, q = ((long long)k * g.nx + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) vwall[c + a] = src ? src[q + a] : 0.0;
  }
  for (int w = 0; w < 2; ++w) {
    const int jf = w == 0 ? 0 : g.H - 1;
    const long long n = ((long long)k * g.H + jf) * g.nx + i;
    double J[3][3], Ji[3][3], det;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + n];
    inv3(J, Ji, det);
    const long long c = (((long long)w * g.nz + k) * g.nx + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      uw[c + a] = (T)(Ji[a][0] * vwall[c] + Ji[a][1] * vwall[c + 1] + Ji[a][2] * vwall[c + 2]);
  }
}

// Chart components J^{-1} v of the plate velocity at the fluid nodes below
// (side 0, row pj - 1) and above (side 1, row pj) the plate's half row; a
// column off the plate takes the velocity of the nearest plate column (the
// diagonal links at the plate's ends).
template <class T>
__global__ __launch_bounds__(BX * BY) void k_plate_velocity(Grid g, const double* __restrict__ jac, double* __restrict__ vplate,
                                                            T* __restrict__ up, int in, const double* __restrict__ src) {
  const int i = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  const int ic = i < g.pi0 ? g.pi0 : (i > g.pi1 ? g.pi1 : i);
  // in: a new plate velocity comes from src (NULL: zero); each column stores
  // its own into the context's copy and reads the nearest plate column's from
  // src, so no thread reads what another writes
  const long long qc = ((long long)k * g.nx + ic) * 3;
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = in ? (src ? src[qc + a] : 0.0) : vplate[qc + a];
  if (in) {
    const long long q = ((long long)k * g.nx + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) vplate[q + a] = src ? src[q + a] : 0.0;
  }
  for (int side = 0; side < 2; ++side) {
    const long long n = ((long long)k * g.H + (g.pj - 1 + side)) * g.nx + i;
    double J[3][3], Ji[3][3], det;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + n];
    inv3(J, Ji, det);
    const long long c = (((long long)side * g.nz + k) * g.nx + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) up[c + a] = (T)(Ji[a][0] * v[0] + Ji[a][1] * v[1] + Ji[a][2] * v[2]);
  }
}

// Inlet velocity in the chart components of the inlet nodes (column 0):
// v_in = J^{-1} u_in per (z, row).
template <class T>
__global__ __launch_bounds__(BX * BY) void k_inlet_velocity(Grid g, const double* __restrict__ jac, const double* __restrict__ uin, T* __restrict__ vin) {
  const int jf = blockIdx.x * BX + threadIdx.x, k = blockIdx.y * BY + threadIdx.y;
  if (jf >= g.H || k >= g.nz) return;
  const long long n = ((long long)k * g.H + jf) * g.nx;
  double J[3][3], Ji[3][3], det;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = jac[(a * 3 + b) * g.N + n];
  inv3(J, Ji, det);
  const long long c = ((long long)k * g.H + jf) * 3;
#pragma unroll
  for (int a = 0; a < 3; ++a) vin[c + a] = (T)(Ji[a][0] * uin[c] + Ji[a][1] * uin[c + 1] + Ji[a][2] * uin[c + 2]);
}

}  // namespace

hipError_t launch_chart_from_disp(Fields& F, hipStream_t s, int which, const double* src) {
  dim3 b(BX, BY), gr((F.g.nx + BX - 1) / BX, (F.g.ny + BY - 1) / BY, F.g.nz);
  if (F.chart_yonly)
    hipLaunchKernelGGL(k_chart_from_disp<false>, gr, b, 0, s, F.g, F.disp, F.dplate, F.chart, which, src);
  else
    hipLaunchKernelGGL(k_chart_from_disp<true>, gr, b, 0, s, F.g, F.disp, F.dplate, F.chart, which, src);
  F.chart_yonly = 1;
  return hipGetLastError();
}

template <class T> hipError_t launch_plate_velocity(Fields& F, hipStream_t s, int in, const double* src) {
  if (!F.g.pj) return hipSuccess;
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_plate_velocity<T>, col_grid(F.g), b, 0, s, F.g, F.jac, F.vplate, (T*)F.up, in, src);
  return hipGetLastError();
}

template <class T> hipError_t launch_geometry(Fields& F, hipStream_t s, const double Fc[3]) {
  const Grid g = F.g;
  dim3 b(BX, BY);
  double* u = F.uext[F.uext_cur];
  // marching grid: x tiles, layer tiles of [jlo, jhi], z chunks
  auto mg = [&](int jlo, int jhi) {
    return dim3((g.nx + BX - 1) / BX, (jhi - jlo + BY) / BY, (g.nz + MZC - 1) / MZC);
  };
  // A chart that moves the nodes along y only has x and z displacements of
  // exactly zero, and so smoothed x and z components of exactly zero: once a
  // buffer holds those zeros, only its y component is written again (the
  // adjoint's chart gradient reads all three components of the smoothed one).
  const bool y = F.chart_yonly;
  if (!y)
    hipLaunchKernelGGL((k_uext<false, true>), ext_grid(g), b, 0, s, g, F.chart, u);
  else if (F.uext_yonly[F.uext_cur])
    hipLaunchKernelGGL((k_uext<true, false>), ext_grid(g), b, 0, s, g, F.chart, u);
  else
    hipLaunchKernelGGL((k_uext<true, true>), ext_grid(g), b, 0, s, g, F.chart, u);
  F.uext_yonly[F.uext_cur] = y;
  if (y && F.vtmp_xz_zero)
    hipLaunchKernelGGL(k_smooth<1>, mg(-2, g.ny + 1), b, 0, s, g, -2, g.ny + 1, u + F.NE, F.vtmp + F.NE);
  else
    hipLaunchKernelGGL(k_smooth<3>, mg(-2, g.ny + 1), b, 0, s, g, -2, g.ny + 1, u, F.vtmp);
  F.vtmp_xz_zero = y;
  // likewise the rows (1, 0, 0) and (0, 0, 1) of J at the fluid nodes
  if (!y)
    hipLaunchKernelGGL((k_jac_metric<false, true>), mg(-1, g.ny), b, 0, s, g, F.vtmp, F.gext, F.jac);
  else if (F.jac_rows_exact)
    hipLaunchKernelGGL((k_jac_metric<true, false>), mg(-1, g.ny), b, 0, s, g, F.vtmp + F.NE, F.gext, F.jac);
  else
    hipLaunchKernelGGL((k_jac_metric<true, true>), mg(-1, g.ny), b, 0, s, g, F.vtmp + F.NE, F.gext, F.jac);
  F.jac_rows_exact = y;
  if (y)
    hipLaunchKernelGGL(k_smooth_gy, mg(0, g.ny - 1), b, 0, s, g, 0, g.ny - 1, F.gext, F.wext);
  else
    hipLaunchKernelGGL(k_smooth<6>, mg(0, g.ny - 1), b, 0, s, g, 0, g.ny - 1, F.gext, F.wext);
  auto* kg = y ? k_geo<T, true> : k_geo<T, false>;
  hipLaunchKernelGGL(kg, mg(1, g.ny - 2), b, 0, s, g, F.wext, F.gext, F.jac, Fc[0], Fc[1], Fc[2], (T*)F.geo);
  return hipGetLastError();
}

template <class T> hipError_t launch_body_force(Fields& F, hipStream_t s, const double Fc[3]) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_body_force<T>, fluid_grid(F.g), b, 0, s, F.g, F.jac, Fc[0], Fc[1], Fc[2], (T*)F.geo);
  return hipGetLastError();
}

template <class T> hipError_t launch_wall_velocity(Fields& F, hipStream_t s, int which, const double* src) {
  dim3 b(BX, BY);
  hipLaunchKernelGGL(k_wall_velocity<T>, col_grid(F.g), b, 0, s, F.g, F.jac, F.vwall, (T*)F.uw, which, src);
  return hipGetLastError();
}

template hipError_t launch_geometry<double>(Fields&, hipStream_t, const double*);
template hipError_t launch_geometry<float>(Fields&, hipStream_t, const double*);
template hipError_t launch_body_force<double>(Fields&, hipStream_t, const double*);
template hipError_t launch_body_force<float>(Fields&, hipStream_t, const double*);
template hipError_t launch_wall_velocity<double>(Fields&, hipStream_t, int, const double*);
template hipError_t launch_wall_velocity<float>(Fields&, hipStream_t, int, const double*);
template <class T> hipError_t launch_inlet_velocity(Fields& F, hipStream_t s) {
  if (!F.g.open) return hipSuccess;
  dim3 b(BX, BY), gr((F.g.H + BX - 1) / BX, (F.g.nz + BY - 1) / BY, 1);
  hipLaunchKernelGGL(k_inlet_velocity<T>, gr, b, 0, s, F.g, F.jac, F.uin, (T*)F.vin);
  return hipGetLastError();
}

template hipError_t launch_inlet_velocity<double>(Fields&, hipStream_t);
template hipError_t launch_inlet_velocity<float>(Fields&, hipStream_t);
template hipError_t launch_plate_velocity<double>(Fields&, hipStream_t, int, const double*);
template hipError_t launch_plate_velocity<float>(Fields&, hipStream_t, int, const double*);

}  // namespace lbm
